// batch.hpp -- many independent bootstrap filters of uneven sizes advanced
// together (one assimilation cycle per graph replay).
//
// Every particle of every instance has a global index g; an instance owns the
// contiguous range [g0, g0 + n).  Per-instance constants (grid, tile
// constants of the Helmholtz scan, pointers to the caller's state) sit in a
// device table.  The forecast runs as one persistent kernel per tile class
// (threads per particle, nodes per thread): its workgroups take (instance,
// particle) items from an atomic queue ordered longest job first.  The
// filter steps (likelihood, weights and ESS, conditional resampling, gathers)
// are batched kernels with one workgroup per instance or per particle; every
// branch of the cycle is taken on the device, so a whole cycle can be
// captured into a HIP graph and replayed, the cycle number being read from
// device memory.
#pragma once

#include "filter.hpp"
#include "model.hpp"

namespace sch {

struct InstDev {
  StepParams P;
  HelmConst K;
  double* m;            // caller state [n][nx]
  double* u;
  double* logw;         // [n] normalised log-weights carried between cycles
  const double* y;      // [cycles][n_obs]: observations of every cycle
  const double* sigma;  // [n_obs]
  uint64_t seed;
  int n, n_obs;
  int64_t g0;           // first global particle index
  int64_t s0;           // first element of the instance in the state scratch
  double thr;           // resampling threshold on the ESS
};

struct BatchDev {
  const InstDev* inst;
  const int* pinst;     // [G] instance of global particle g
  int G, n_inst, n_steps, n_modes;
  const unsigned int* cycle;  // device cycle counter
  double* dW;           // [G][n_steps][n_modes]
  double* phi;          // [G]
  double* w;            // [G]
  double* theta;        // [n_inst]
  double* dtheta;       // [n_inst]
  double* ess;          // [n_inst]
  double* u0;           // [n_inst]
  int* idx;             // [G] (local indices)
  int* degenerate;      // [n_inst]
  int* resampled;       // [n_inst] resamplings counted over the run
  int* status;          // [G] first failure over the run
  unsigned long long* cum;    // [G]
  double* scratch;      // state scratch, sum of n * nx per instance
  unsigned long long* acc;    // [1] Picard iterations
};

// Forecast increments of every particle: counter (p, cycle * n_steps + n,
// pair | FORECAST << 24, 0) under the instance's seed, as sch_draw_increments.
__global__ void k_batch_draw(BatchDev B) {
  const int n_pairs = (B.n_modes + 1) / 2;
  const int64_t total = static_cast<int64_t>(B.G) * B.n_steps * n_pairs;
  const uint32_t step0 = *B.cycle * static_cast<uint32_t>(B.n_steps);
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < total;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int kk = static_cast<int>(i % n_pairs);
    const int64_t gn = i / n_pairs;
    const int n = static_cast<int>(gn % B.n_steps);
    const int g = static_cast<int>(gn / B.n_steps);
    const InstDev& D = B.inst[B.pinst[g]];
    const int p = static_cast<int>(g - D.g0);
    double z0, z1;
    normal2(D.seed, static_cast<uint32_t>(p), step0 + static_cast<uint32_t>(n),
            static_cast<uint32_t>(kk) | (SCH_TAG_FORECAST << 24), 0u, z0, z1);
    const double sdt = sqrt(D.P.dt);
    double* row = B.dW + gn * B.n_modes;
    row[2 * kk] = sdt * z0;
    if (2 * kk + 1 < B.n_modes) row[2 * kk + 1] = sdt * z1;
  }
}

// Persistent forecast kernel of one tile class: items[0..n_items) are global
// particle indices, longest job first; *queue must be zero at launch.  Every
// workgroup leaves once the queue is exhausted.
template <int PMAX, int NT>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2))) k_batch_window(BatchDev B, const int* items, int n_items,
                                                     unsigned int* queue) {
  __shared__ RowLds<NT> L;
  __shared__ AuxLds<PMAX, NT> X;
  __shared__ int s_item;
  const int t = threadIdx.x;
  // Work fetch without a lane-divergent branch: a divergent `if (t == 0)`
  // at the top of this loop lets the compiler split the loop by lanes
  // (thread 0 taken out to fetch while the rest of its wavefront re-runs the
  // old item, forever).  Wavefront 0 takes a uniform branch, all its lanes
  // join one atomic that adds 1 (lane 0's term), and the index lives in
  // scalar registers.
  const bool wave0 = __builtin_amdgcn_readfirstlane(t) == 0;
  for (;;) {
    if (wave0) {
      const unsigned v = atomicAdd(queue, t == 0 ? 1u : 0u);
      s_item = static_cast<int>(__builtin_amdgcn_readfirstlane(v));
    }
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();
    if (it >= n_items) break;
    const int g = items[it];
    const InstDev& D = B.inst[B.pinst[g]];
    const StepParams P = D.P;
    const HelmConst K = D.K;
    const int p = static_cast<int>(g - D.g0);
    const Chunk ch = chunk_of<NT>(P.nx, t);
    double* mp = D.m + static_cast<size_t>(p) * P.nx;
    double* up = D.u + static_cast<size_t>(p) * P.nx;
    double m[PMAX], u[PMAX];
    load_chunk<PMAX, false>(mp, ch, m);
    load_chunk<PMAX, false>(up, ch, u);
    const double* dW = B.dW + static_cast<size_t>(g) * B.n_steps * B.n_modes;
    const int Q = B.n_modes;
    auto inc = [&](int n, int q) { return dW[n * Q + q]; };
    int iters = 0;
    Parity par;
    const int st = run_window<PMAX, NT, false>(P, K, modes_noise<PMAX, false>(P, ch, inc), B.n_steps,
                                                 m, u, ch, L, X, t, par, iters);
    store_chunk<PMAX, false>(mp, ch, m);
    store_chunk<PMAX, false>(up, ch, u);
    if (t == 0) {
      if (st != SCH_OK && B.status[g] == SCH_OK) B.status[g] = st;
      // a failed window marks the particle for the likelihood (zero weight)
      B.phi[g] = st == SCH_OK ? 0.0 : INFINITY;
      atomicAdd(B.acc, static_cast<unsigned long long>(iters));
    }
  }
}

// Negative log-likelihood of every particle against its instance's
// observations of the current cycle (one wavefront per particle).
__global__ void __launch_bounds__(kWave) k_batch_loglik(BatchDev B) {
  const int g = blockIdx.x;
  const InstDev& D = B.inst[B.pinst[g]];
  const int p = static_cast<int>(g - D.g0);
  const int nx = D.P.nx, n_obs = D.n_obs;
  const double* up = D.u + static_cast<size_t>(p) * nx;
  const double* y = D.y + static_cast<size_t>(*B.cycle) * n_obs;
  if (!(B.phi[g] < INFINITY)) return;  // the particle's window failed this cycle
  double acc = 0.0;
  for (int j = threadIdx.x; j < n_obs; j += kWave) {
    const double e = (p1_at(up, nx, n_obs, j) - y[j]) / D.sigma[j];
    acc += e * e;
  }
  acc = wave_sum(acc);
  if (threadIdx.x == 0) {
    const double v = 0.5 * acc;
    B.phi[g] = isfinite(v) ? v : INFINITY;
  }
}

// Per instance: weights from the carried log-weights and the likelihood,
// ESS, and the resampling uniform (counter (0, cycle, RESAMPLE << 24, 0)).
__global__ void __launch_bounds__(kTB) k_batch_weights(BatchDev B) {
  __shared__ TemperLds L;
  const int i = blockIdx.x;
  const InstDev& D = B.inst[i];
  if (threadIdx.x == 0) B.theta[i] = 0.0;
  __syncthreads();
  temper_body(D.n, B.phi + D.g0, D.logw, B.theta + i, 0.0, 0, B.dtheta + i, B.w + D.g0, D.logw,
              B.ess + i, L);
  if (threadIdx.x == 0) B.u0[i] = uniform1(D.seed, 0u, *B.cycle, SCH_TAG_RESAMPLE << 24, 0u);
}

// Per instance: systematic resampling when ESS < threshold (identity
// indices otherwise).
__global__ void __launch_bounds__(kTB) k_batch_resample(BatchDev B) {
  __shared__ ResampleLds L;
  const int i = blockIdx.x;
  const InstDev& D = B.inst[i];
  resample_body(D.n, B.w + D.g0, B.u0 + i, B.ess + i, D.thr, B.idx + D.g0, B.degenerate + i,
                B.cum + D.g0, L);
  if (threadIdx.x == 0 && !(B.ess[i] >= D.thr)) B.resampled[i] += 1;
}

// Gather of the resampled instances, one workgroup per particle: scratch row
// p = state row idx[p] (phase 0), then back into the caller's arrays with the
// log-weights reset (phase 1).  Instances that kept their particles are
// skipped.
__global__ void k_batch_gather(BatchDev B, int phase) {
  const int g = blockIdx.x;
  const int i = B.pinst[g];
  const InstDev& D = B.inst[i];
  if (B.ess[i] >= D.thr) return;
  const int p = static_cast<int>(g - D.g0);
  const int nx = D.P.nx;
  double* sm = B.scratch + D.s0 + static_cast<int64_t>(p) * 2 * nx;
  if (phase == 0) {
    const int r = B.idx[g];
    const double* mr = D.m + static_cast<int64_t>(r) * nx;
    const double* ur = D.u + static_cast<int64_t>(r) * nx;
    for (int k = threadIdx.x; k < nx; k += blockDim.x) {
      sm[k] = mr[k];
      sm[nx + k] = ur[k];
    }
  } else {
    double* mp = D.m + static_cast<int64_t>(p) * nx;
    double* up = D.u + static_cast<int64_t>(p) * nx;
    for (int k = threadIdx.x; k < nx; k += blockDim.x) {
      mp[k] = sm[k];
      up[k] = sm[nx + k];
    }
    if (threadIdx.x == 0) D.logw[p] = 0.0;
  }
}

__global__ void k_batch_next_cycle(unsigned int* cycle) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *cycle += 1u;
}

__global__ void k_fill_u32(unsigned int* p, unsigned int v, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = v;
}

}  // namespace sch
