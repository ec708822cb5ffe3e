// model.hpp -- kernels of the SCH forward model on gfx950: one workgroup per
// particle, the particle's row of nx nodes split in register chunks over the
// workgroup's threads, every linear system solved with cyclic_solve().
#pragma once

#include "device.hpp"

namespace sch {

// Per-call constants of the P1 / implicit-midpoint discretisation.
struct StepParams {
  int nx, n_modes, picard_max;
  double h, dt, tol;
  double a_off, a_diag;  // constant parts of the step matrix rows:
                         // h/6 - mu dt/(2h) and 2h/3 + mu dt/h
  double h_off, h_diag;  // Helmholtz rows: h/6 - alpha^2/h and 2h/3 + 2 alpha^2/h
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
  const double a2 = md.alpha * md.alpha;
  P.h_off = P.h / 6.0 - a2 / P.h;
  P.h_diag = 2.0 * P.h / 3.0 + 2.0 * a2 / P.h;
  P.xi = md.xi;
  return P;
}

// Mass-matrix product (M v)_j = h/6 v_{j-1} + 2h/3 v_j + h/6 v_{j+1} on a chunk.
template <int PMAX, int NT, bool FULL>
__device__ __forceinline__ void mass_apply(const double (&v)[PMAX], double (&out)[PMAX], double h,
                                           int cnt, RowLds<NT>& L, int t, double scale) {
  double hl, hr;
  halo<PMAX, NT, FULL>(v, cnt, L, t, hl, hr);
  const double c1 = scale * h / 6.0, c0 = scale * 2.0 * h / 3.0;
#pragma unroll
  for (int j = 0; j < PMAX; ++j)
    out[j] = c1 * (left_of<PMAX, FULL>(v, j, hl) + right_of<PMAX, FULL>(v, j, cnt, hr)) + c0 * v[j];
}

// u = H^{-1} M m on a chunk (Helmholtz relation, first line of eq. fde1).
template <int PMAX, int NT, bool FULL>
__device__ __forceinline__ void helmholtz(const StepParams& P, const double (&m)[PMAX],
                                          double (&u)[PMAX], int cnt, RowLds<NT>& L, int t) {
  double r[PMAX];
  mass_apply<PMAX, NT, FULL>(m, r, P.h, cnt, L, t, 1.0);
  const double ho = P.h_off, hd = P.h_diag;
  auto rowH = [&](int, double& a, double& b, double& c) {
    a = ho;
    b = hd;
    c = ho;
  };
  cyclic_solve<PMAX, NT, FULL>(rowH, r, u, cnt, L, t);
}

// One assimilation window of n_steps implicit-midpoint steps (eq. fde1) for
// the particle whose chunk is held in m, u.  inc(n, q) returns the noise
// increment dW^n_q (+ dLambda^n_q) of step n, mode q.
//
// Each step solves  A(dv) s = 2 M m^n  for s = m^n + m^{n+1}, with
//   A(dv) = M + (mu dt/2) K + (1/2) C(dv),  dv = dt (u^n + u*)/2 + dU^n,
// by Picard iteration on u* (u* = u^n initially, then u* = H^{-1} M m*), until
// the max-norm change of m* is at most tol * max|m*|.  Rows of A at node i:
//   a_i = h/6 - mu dt/(2h) - dv_{i-1}/4
//   b_i = 2h/3 + mu dt/h + (dv_{i+1} - dv_{i-1})/4
//   c_i = h/6 - mu dt/(2h) + dv_{i+1}/4
// (the exact P1 integrals of the advective terms of eq. fde1).
// Returns SCH_OK or the status of the first failing step; on non-convergence
// the last iterate is kept, on a non-finite iterate the step's input is kept.
template <int PMAX, int NT, bool FULL, class IncF>
__device__ int run_window(const StepParams& P, IncF inc, int n_steps, double (&m)[PMAX],
                          double (&u)[PMAX], const Chunk& ch, RowLds<NT>& L, int t, int& iters) {
  const int cnt = ch.cnt;
  const double hdt = 0.5 * P.dt;
  for (int n = 0; n < n_steps; ++n) {
    // dU^n + dt/2 u^n, the explicit part of dv
    double dUp[PMAX];
#pragma unroll
    for (int j = 0; j < PMAX; ++j) dUp[j] = hdt * u[j];
    for (int q = 0; q < P.n_modes; ++q) {
      const double w = inc(n, q);
      const double* xq = P.xi + static_cast<size_t>(q) * P.nx + ch.start;
#pragma unroll
      for (int j = 0; j < PMAX; ++j)
        if (FULL || j < cnt) dUp[j] += xq[j] * w;
    }
    double f[PMAX];
    mass_apply<PMAX, NT, FULL>(m, f, P.h, cnt, L, t, 2.0);

    double us[PMAX], mp[PMAX], ms[PMAX];
#pragma unroll
    for (int j = 0; j < PMAX; ++j) {
      us[j] = u[j];
      mp[j] = m[j];
    }
    int status = SCH_E_NONCONVERGED, k = 1;
    for (; k <= P.picard_max; ++k) {
      double dv[PMAX];
#pragma unroll
      for (int j = 0; j < PMAX; ++j) dv[j] = hdt * us[j] + dUp[j];
      double vl, vr;
      halo<PMAX, NT, FULL>(dv, cnt, L, t, vl, vr);
      const double ao = P.a_off, ad = P.a_diag;
      auto rowA = [&](int j, double& a, double& b, double& c) {
        const double vm = left_of<PMAX, FULL>(dv, j, vl);
        const double vp = right_of<PMAX, FULL>(dv, j, cnt, vr);
        a = ao - 0.25 * vm;
        b = ad + 0.25 * (vp - vm);
        c = ao + 0.25 * vp;
      };
      cyclic_solve<PMAX, NT, FULL>(rowA, f, ms, cnt, L, t);
#pragma unroll
      for (int j = 0; j < PMAX; ++j) ms[j] -= m[j];
      helmholtz<PMAX, NT, FULL>(P, ms, us, cnt, L, t);
      double diff = 0.0, scale = 0.0;
      int bad = 0;
#pragma unroll
      for (int j = 0; j < PMAX; ++j) {
        if (FULL || j < cnt) {
          diff = fmax(diff, fabs(ms[j] - mp[j]));
          scale = fmax(scale, fabs(ms[j]));
          bad |= !isfinite(ms[j]) || !isfinite(us[j]);
        }
        mp[j] = ms[j];
      }
      block_max2_or<NT>(diff, scale, bad, L, t);
      if (bad) {
        status = SCH_E_NONFINITE;
        break;
      }
      if (diff <= P.tol * scale) {
        status = SCH_OK;
        break;
      }
    }
    iters += k > P.picard_max ? P.picard_max : k;
    if (status == SCH_E_NONFINITE) return status;
#pragma unroll
    for (int j = 0; j < PMAX; ++j) {
      m[j] = ms[j];
      u[j] = us[j];
    }
    if (status != SCH_OK) return status;
  }
  return SCH_OK;
}

// Negative log-likelihood of the particle's velocity chunk (eq. loglikeq):
// each thread takes the observation points that fall in its own cells.
template <int PMAX, int NT, bool FULL>
__device__ double block_nll(const double (&u)[PMAX], const Chunk& ch, int nx, int n_obs,
                            const double* y, const double* sigma, RowLds<NT>& L, int t) {
  double hl, hr;
  halo<PMAX, NT, FULL>(u, ch.cnt, L, t, hl, hr);
  double acc = 0.0;
#pragma unroll
  for (int j = 0; j < PMAX; ++j) {
    if (!FULL && j >= ch.cnt) continue;
    const int64_t node = ch.start + j;
    const int64_t jlo = (node * n_obs + nx - 1) / nx;
    const int64_t jhi = ((node + 1) * n_obs + nx - 1) / nx;
    const double ur = right_of<PMAX, FULL>(u, j, ch.cnt, hr);
    for (int64_t o = jlo; o < jhi; ++o) {
      const double r = static_cast<double>((o * nx) % n_obs) / static_cast<double>(n_obs);
      const double pu = (1.0 - r) * u[j] + r * ur;
      const double e = (pu - y[o]) / sigma[o];
      acc += e * e;
    }
  }
  return 0.5 * block_sum<NT>(acc, L, t);
}

template <int PMAX, bool FULL>
__device__ __forceinline__ void load_chunk(const double* g, const Chunk& ch, double (&v)[PMAX]) {
#pragma unroll
  for (int j = 0; j < PMAX; ++j) v[j] = (FULL || j < ch.cnt) ? g[ch.start + j] : 0.0;
}
template <int PMAX, bool FULL>
__device__ __forceinline__ void store_chunk(double* g, const Chunk& ch, const double (&v)[PMAX]) {
#pragma unroll
  for (int j = 0; j < PMAX; ++j)
    if (FULL || j < ch.cnt) g[ch.start + j] = v[j];
}

// ---------------------------------------------------------------------------
// Kernels.
// ---------------------------------------------------------------------------
struct WindowArgs {
  StepParams P;
  int n_steps;
  double* m;
  double* u;
  const double* dW;
  const double* dLam;
  int* status;
  int* iters;
  unsigned long long* iters_acc;  // optional device accumulator
};

template <int PMAX, int NT, bool FULL>
__global__ void __launch_bounds__(NT) k_window(const WindowArgs A) {
  __shared__ RowLds<NT> L;
  const int p = blockIdx.x, t = threadIdx.x;
  const Chunk ch = chunk_of<NT>(A.P.nx, t);
  double* mp = A.m + static_cast<size_t>(p) * A.P.nx;
  double* up = A.u + static_cast<size_t>(p) * A.P.nx;
  double m[PMAX], u[PMAX];
  load_chunk<PMAX, FULL>(mp, ch, m);
  load_chunk<PMAX, FULL>(up, ch, u);
  const int Q = A.P.n_modes;
  const double* dW = A.dW + static_cast<size_t>(p) * A.n_steps * Q;
  const double* dL = A.dLam ? A.dLam + static_cast<size_t>(p) * A.n_steps * Q : nullptr;
  auto inc = [&](int n, int q) {
    double w = dW[n * Q + q];
    if (dL) w += dL[n * Q + q];
    return w;
  };
  int iters = 0;
  const int st = run_window<PMAX, NT, FULL>(A.P, inc, A.n_steps, m, u, ch, L, t, iters);
  store_chunk<PMAX, FULL>(mp, ch, m);
  store_chunk<PMAX, FULL>(up, ch, u);
  if (t == 0) {
    if (A.status) A.status[p] = st;
    if (A.iters) A.iters[p] = iters;
    if (A.iters_acc) atomicAdd(A.iters_acc, static_cast<unsigned long long>(iters));
  }
}

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
  uint64_t seed;
  uint32_t cycle, temper_k;
};

template <int PMAX, int NT, bool FULL>
__global__ void __launch_bounds__(NT) k_jitter(const JitterArgs A) {
  __shared__ RowLds<NT> L;
  extern __shared__ double dyn[];  // [2][n_steps][n_modes]: current increments, proposal
  const int p = blockIdx.x, t = threadIdx.x;
  const int nx = A.P.nx, Q = A.P.n_modes, S = A.n_steps;
  const Chunk ch = chunk_of<NT>(nx, t);
  double* cur = dyn;
  double* prop = dyn + S * Q;
  double m0[PMAX], u0[PMAX];
  load_chunk<PMAX, FULL>(A.m0 + static_cast<size_t>(p) * nx, ch, m0);
  load_chunk<PMAX, FULL>(A.u0 + static_cast<size_t>(p) * nx, ch, u0);
  double* dWp = A.dW + static_cast<size_t>(p) * S * Q;
  for (int i = t; i < S * Q; i += NT) cur[i] = dWp[i];
  double phi = A.phi[p];
  const double theta = *A.theta;
  const double srho = sqrt(1.0 - A.rho * A.rho), sdt = sqrt(A.P.dt);
  const int n_pairs = (Q + 1) / 2;
  int acc = 0, iters = 0;
  __syncthreads();
  for (int j = 0; j < A.n_jitter; ++j) {
    const uint32_t w3 = (A.temper_k << 16) | static_cast<uint32_t>(j);
    for (int i = t; i < S * n_pairs; i += NT) {
      const int n = i / n_pairs, kk = i - n * n_pairs;
      double z0, z1;
      normal2(A.seed, static_cast<uint32_t>(p), A.cycle * static_cast<uint32_t>(S) + n,
              static_cast<uint32_t>(kk) | (SCH_TAG_PCN << 24), w3, z0, z1);
      const int q0 = 2 * kk;
      prop[n * Q + q0] = A.rho * cur[n * Q + q0] + srho * (sdt * z0);
      if (q0 + 1 < Q) prop[n * Q + q0 + 1] = A.rho * cur[n * Q + q0 + 1] + srho * (sdt * z1);
    }
    __syncthreads();
    double m[PMAX], u[PMAX];
#pragma unroll
    for (int q = 0; q < PMAX; ++q) {
      m[q] = m0[q];
      u[q] = u0[q];
    }
    auto inc = [&](int n, int q) { return prop[n * Q + q]; };
    const int st = run_window<PMAX, NT, FULL>(A.P, inc, S, m, u, ch, L, t, iters);
    double phin = block_nll<PMAX, NT, FULL>(u, ch, nx, A.n_obs, A.y, A.sigma, L, t);
    if (st != SCH_OK || !isfinite(phin)) phin = INFINITY;
    const double v = uniform1(A.seed, static_cast<uint32_t>(p), A.cycle, SCH_TAG_ACCEPT << 24, w3);
    bool accept;
    if (!(phin < INFINITY)) {
      accept = false;
    } else {
      const double logr = theta * (phi - phin);
      accept = logr >= 0.0 ? true : (v < exp(logr));
    }
    if (accept) {
      for (int i = t; i < S * Q; i += NT) cur[i] = prop[i];
      store_chunk<PMAX, FULL>(A.m_end + static_cast<size_t>(p) * nx, ch, m);
      store_chunk<PMAX, FULL>(A.u_end + static_cast<size_t>(p) * nx, ch, u);
      phi = phin;
      ++acc;
    }
    __syncthreads();
  }
  if (acc > 0)
    for (int i = t; i < S * Q; i += NT) dWp[i] = cur[i];
  if (t == 0) {
    A.phi[p] = phi;
    if (A.n_accept) A.n_accept[p] = acc;
    if (A.accept_acc) atomicAdd(A.accept_acc, static_cast<unsigned long long>(acc));
    if (A.iters_acc) atomicAdd(A.iters_acc, static_cast<unsigned long long>(iters));
  }
}

// u = H^{-1} M m (mode 0) or m = M^{-1} H u (mode 1) for every particle.
struct HelmArgs {
  StepParams P;
  const double* in;
  double* out;
  int mode;
};

template <int PMAX, int NT, bool FULL>
__global__ void __launch_bounds__(NT) k_helmholtz(const HelmArgs A) {
  __shared__ RowLds<NT> L;
  const int p = blockIdx.x, t = threadIdx.x;
  const Chunk ch = chunk_of<NT>(A.P.nx, t);
  double v[PMAX], o[PMAX];
  load_chunk<PMAX, FULL>(A.in + static_cast<size_t>(p) * A.P.nx, ch, v);
  if (A.mode == 0) {
    helmholtz<PMAX, NT, FULL>(A.P, v, o, ch.cnt, L, t);
  } else {
    // right-hand side H u = M u + alpha^2 K u, then the mass solve
    double hl, hr;
    halo<PMAX, NT, FULL>(v, ch.cnt, L, t, hl, hr);
    double r[PMAX];
#pragma unroll
    for (int j = 0; j < PMAX; ++j)
      r[j] = A.P.h_off * (left_of<PMAX, FULL>(v, j, hl) + right_of<PMAX, FULL>(v, j, ch.cnt, hr)) +
             A.P.h_diag * v[j];
    const double mo = A.P.h / 6.0, md = 2.0 * A.P.h / 3.0;
    auto rowM = [&](int, double& a, double& b, double& c) {
      a = mo;
      b = md;
      c = mo;
    };
    cyclic_solve<PMAX, NT, FULL>(rowM, r, o, ch.cnt, L, t);
  }
  store_chunk<PMAX, FULL>(A.out + static_cast<size_t>(p) * A.P.nx, ch, o);
}

}  // namespace sch
