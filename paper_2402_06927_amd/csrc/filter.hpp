// filter.hpp -- particle-filter kernels on gfx950: noise draws, observation
// and likelihood, weights / ESS / tempering, systematic resampling, gathers.
#pragma once

#include "device.hpp"

namespace sch {

// dW[p][n][q] = sqrt(dt) z, one Philox block per (particle, step, mode pair).
__global__ void k_draw_increments(uint64_t seed, uint32_t step0, uint32_t tag, uint32_t word3,
                                  int n_particles, int n_steps, int n_modes, double sdt,
                                  double* dW) {
  const int n_pairs = (n_modes + 1) / 2;
  const int64_t total = static_cast<int64_t>(n_particles) * n_steps * n_pairs;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < total;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int kk = static_cast<int>(i % n_pairs);
    const int64_t pn = i / n_pairs;
    const int n = static_cast<int>(pn % n_steps);
    const int p = static_cast<int>(pn / n_steps);
    double z0, z1;
    normal2(seed, static_cast<uint32_t>(p), step0 + static_cast<uint32_t>(n),
            static_cast<uint32_t>(kk) | (tag << 24), word3, z0, z1);
    double* row = dW + pn * n_modes;
    row[2 * kk] = sdt * z0;
    if (2 * kk + 1 < n_modes) row[2 * kk + 1] = sdt * z1;
  }
}

// Raw Philox blocks: out[i] = philox(ctr[i], seed).
__global__ void k_philox_blocks(uint64_t seed, int n, const uint32_t* ctr, uint32_t* out) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const Ctr4 r = philox10(Ctr4{{ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]}}, seed);
#pragma unroll
    for (int k = 0; k < 4; ++k) out[4 * i + k] = r.w[k];
  }
}

// Random numbers of n_jitter pCN moves (section 3.1.2): zeta[j][p][n][q] =
// sqrt(dt) z with z from the PCN-tagged block (p, step0 + n, pair | tag << 24,
// word3 | j), and the acceptance uniform vacc[j][p] from the ACCEPT-tagged
// block (p, cycle, tag << 24, word3 | j).
__global__ void k_draw_pcn(uint64_t seed, uint32_t step0, uint32_t cycle, uint32_t word3,
                           int n_jitter, int n_particles, int n_steps, int n_modes, double sdt,
                           double* zeta, double* vacc) {
  const int n_pairs = (n_modes + 1) / 2;
  const int64_t per = static_cast<int64_t>(n_particles) * n_steps * n_pairs;
  const int64_t total = per * n_jitter;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < total;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int j = static_cast<int>(i / per);
    const int64_t r = i - j * per;
    const int kk = static_cast<int>(r % n_pairs);
    const int64_t pn = r / n_pairs;
    const int n = static_cast<int>(pn % n_steps);
    const int p = static_cast<int>(pn / n_steps);
    const uint32_t w3 = word3 | static_cast<uint32_t>(j);
    double z0, z1;
    normal2(seed, static_cast<uint32_t>(p), step0 + static_cast<uint32_t>(n),
            static_cast<uint32_t>(kk) | (SCH_TAG_PCN << 24), w3, z0, z1);
    double* row = zeta + (static_cast<int64_t>(j) * n_particles * n_steps + pn) * n_modes;
    row[2 * kk] = sdt * z0;
    if (2 * kk + 1 < n_modes) row[2 * kk + 1] = sdt * z1;
    if (n == 0 && kk == 0)
      vacc[static_cast<int64_t>(j) * n_particles + p] =
          uniform1(seed, static_cast<uint32_t>(p), cycle, SCH_TAG_ACCEPT << 24, w3);
  }
}

// One uniform in [0,1) into a device scalar.
__global__ void k_draw_uniform(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                               double* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *out = uniform1(seed, c0, c1, c2, c3);
}

// P1 point evaluation at x_j = j L / n_obs, one wavefront per particle.
__device__ __forceinline__ double p1_at(const double* u, int nx, int n_obs, int j) {
  const int64_t num = static_cast<int64_t>(j) * nx;
  const int e = static_cast<int>(num / n_obs);
  const double r = static_cast<double>(num % n_obs) / static_cast<double>(n_obs);
  const int e1 = e + 1 == nx ? 0 : e + 1;
  return (1.0 - r) * u[e] + r * u[e1];
}

__global__ void __launch_bounds__(kWave) k_observe(int nx, int n_obs, const double* u,
                                                   double* out) {
  const int p = blockIdx.x;
  const double* up = u + static_cast<size_t>(p) * nx;
  for (int j = threadIdx.x; j < n_obs; j += kWave)
    out[static_cast<size_t>(p) * n_obs + j] = p1_at(up, nx, n_obs, j);
}

__global__ void __launch_bounds__(kWave) k_loglik(int nx, int n_obs, const double* u,
                                                  const double* y, const double* sigma,
                                                  double* phi) {
  const int p = blockIdx.x;
  const double* up = u + static_cast<size_t>(p) * nx;
  double acc = 0.0;
  for (int j = threadIdx.x; j < n_obs; j += kWave) {
    const double e = (p1_at(up, nx, n_obs, j) - y[j]) / sigma[j];
    acc += e * e;
  }
  acc = wave_sum(acc);
  if (threadIdx.x == 0) {
    const double v = 0.5 * acc;
    phi[p] = isfinite(v) ? v : INFINITY;
  }
}

// ---------------------------------------------------------------------------
// Weights, ESS and adaptive tempering in one workgroup of kTB threads.
// ---------------------------------------------------------------------------
constexpr int kTB = 1024;

struct TemperLds {
  double red[2][kTB / kWave];
};

__device__ __forceinline__ double tb_reduce_max(double v, TemperLds& L) {
  v = wave_max(v);
  const int w = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0) L.red[0][w] = v;
  __syncthreads();
  double r = L.red[0][0];
  for (int i = 1; i < kTB / kWave; ++i) r = fmax(r, L.red[0][i]);
  __syncthreads();
  return r;
}

__device__ __forceinline__ void tb_reduce_sum2(double& a, double& b, TemperLds& L) {
  a = wave_sum(a);
  b = wave_sum(b);
  const int w = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0) {
    L.red[0][w] = a;
    L.red[1][w] = b;
  }
  __syncthreads();
  double ra = 0.0, rb = 0.0;
  for (int i = 0; i < kTB / kWave; ++i) {
    ra += L.red[0][i];
    rb += L.red[1][i];
  }
  a = ra;
  b = rb;
  __syncthreads();
}

// exponent s_p = extra_p - beta phi_p (a NaN or -inf exponent gives weight 0)
__device__ __forceinline__ double log_weight(double phi, double extra, double beta) {
  double s;
  if (beta == 0.0)
    s = extra;
  else if (isnan(phi))
    s = -INFINITY;
  else
    s = extra - beta * phi;
  return isnan(s) ? -INFINITY : s;
}

// ESS at beta; also returns the max exponent and the sum of exp(s - smax).
__device__ double ess_at(int n, const double* phi, const double* extra, double beta,
                         double& smax, double& tot, TemperLds& L) {
  double mx = -INFINITY;
  for (int p = threadIdx.x; p < n; p += kTB)
    mx = fmax(mx, log_weight(phi[p], extra ? extra[p] : 0.0, beta));
  smax = tb_reduce_max(mx, L);
  if (!(smax > -INFINITY)) {
    tot = 0.0;
    return 0.0;
  }
  double s1 = 0.0, s2 = 0.0;
  for (int p = threadIdx.x; p < n; p += kTB) {
    const double e = exp(log_weight(phi[p], extra ? extra[p] : 0.0, beta) - smax);
    s1 += e;
    s2 += e * e;
  }
  tb_reduce_sum2(s1, s2, L);
  tot = s1;
  return s1 * s1 / s2;
}

// Body of k_temper for one workgroup of kTB threads (also used per
// instance by the batched runner).
__device__ void temper_body(int n, const double* phi, const double* extra, double* theta_io,
                            double thr, int n_bisect, double* dtheta_out, double* w,
                            double* logw_out, double* ess_out, TemperLds& L) {
  const double theta = *theta_io;
  const double rem = 1.0 - theta;
  double smax, tot;
  double e = ess_at(n, phi, extra, rem, smax, tot, L);
  double pick = rem;
  if (n_bisect > 0 && !(e >= thr)) {
    double lo = 0.0, hi = rem;
    for (int k = 0; k < n_bisect; ++k) {
      const double mid = 0.5 * (lo + hi);
      const double em = ess_at(n, phi, extra, mid, smax, tot, L);
      if (em >= thr)
        lo = mid;
      else
        hi = mid;
    }
    pick = lo > 0.0 ? lo : hi;
    e = ess_at(n, phi, extra, pick, smax, tot, L);
  }
  const bool dead = !(smax > -INFINITY);
  const double ltot = dead ? 0.0 : log(tot);
  for (int p = threadIdx.x; p < n; p += kTB) {
    const double s = log_weight(phi[p], extra ? extra[p] : 0.0, pick);
    w[p] = dead ? 0.0 : exp(s - smax) / tot;
    if (logw_out) logw_out[p] = dead ? -INFINITY : (s - smax) - ltot;
  }
  __syncthreads();  // every thread has read *theta_io
  if (threadIdx.x == 0) {
    *dtheta_out = pick;
    *ess_out = e;
    *theta_io = (pick == rem) ? 1.0 : theta + pick;
  }
}

__global__ void __launch_bounds__(kTB) k_temper(int n, const double* phi, const double* extra,
                                                double* theta_io, double thr, int n_bisect,
                                                double* dtheta_out, double* w, double* logw_out,
                                                double* ess_out) {
  __shared__ TemperLds L;
  temper_body(n, phi, extra, theta_io, thr, n_bisect, dtheta_out, w, logw_out, ess_out, L);
}

// ---------------------------------------------------------------------------
// Integer-exact systematic resampling in one workgroup of kTB threads.
// cum (workspace, uint64 [n]) receives the prefix sums of the quantised weights.
// ---------------------------------------------------------------------------
struct ResampleLds {
  double red[kTB / kWave];
  unsigned long long part[kTB];
  int flag;
};

// T_j = ((j + u0) * Q) / n, each operation rounded once (no contraction).
__device__ __forceinline__ double systematic_point(int j, double u0, double Q, int n) {
  double t = __dadd_rn(static_cast<double>(j), u0);
  t = __dmul_rn(t, Q);
  return __ddiv_rn(t, static_cast<double>(n));
}

// Body of k_resample for one workgroup of kTB threads (also used per
// instance by the batched runner).
__device__ void resample_body(int n, const double* w, const double* u0p, const double* cond_ess,
                              double cond_thr, int* idx, int* degenerate,
                              unsigned long long* cum, ResampleLds& L) {
  const int t = threadIdx.x;
  if (cond_ess && *cond_ess >= cond_thr) {
    for (int j = t; j < n; j += kTB) idx[j] = j;
    return;
  }
  // max weight and validity
  double mx = 0.0;
  int bad = 0;
  for (int p = t; p < n; p += kTB) {
    const double v = w[p];
    if (!(v >= 0.0) || isinf(v)) bad = 1;
    mx = fmax(mx, v);
  }
  mx = wave_max(mx);
  bad = wave_or(bad);
  if (t == 0) L.flag = 0;
  __syncthreads();
  if ((t & (kWave - 1)) == 0) {
    L.red[t / kWave] = mx;
    if (bad) atomicOr(&L.flag, 1);
  }
  __syncthreads();
  double wmax = L.red[0];
  for (int i = 1; i < kTB / kWave; ++i) wmax = fmax(wmax, L.red[i]);
  if (L.flag || !(wmax > 0.0)) {
    for (int j = t; j < n; j += kTB) idx[j] = j;
    if (t == 0 && degenerate) *degenerate = 1;
    return;
  }
  int e;
  frexp(wmax, &e);
  int b = 0;
  while ((1LL << b) < n) ++b;
  const int sh = 51 - b - e;
  // contiguous block of particles per thread: local sums, then a scan of the
  // per-thread totals
  const int per = (n + kTB - 1) / kTB;
  const int lo = t * per, hi = min(n, lo + per);
  unsigned long long s = 0;
  for (int p = lo; p < hi; ++p) s += static_cast<unsigned long long>(floor(ldexp(w[p], sh)));
  L.part[t] = s;
  __syncthreads();
  for (int d = 1; d < kTB; d <<= 1) {
    const unsigned long long add = t >= d ? L.part[t - d] : 0ull;
    __syncthreads();
    L.part[t] += add;
    __syncthreads();
  }
  unsigned long long run = t > 0 ? L.part[t - 1] : 0ull;
  for (int p = lo; p < hi; ++p) {
    run += static_cast<unsigned long long>(floor(ldexp(w[p], sh)));
    cum[p] = run;
  }
  const unsigned long long Qi = L.part[kTB - 1];
  __threadfence_block();
  __syncthreads();
  if (Qi == 0ull) {
    for (int j = t; j < n; j += kTB) idx[j] = j;
    if (t == 0 && degenerate) *degenerate = 1;
    return;
  }
  const double Q = static_cast<double>(Qi);
  const double u0 = *u0p;
  for (int j = t; j < n; j += kTB) {
    const double T = systematic_point(j, u0, Q, n);
    // first p with cum[p] > T
    int a = 0, c = n;
    while (a < c) {
      const int mid = (a + c) >> 1;
      if (static_cast<double>(cum[mid]) > T)
        c = mid;
      else
        a = mid + 1;
    }
    idx[j] = a < n ? a : n - 1;
  }
}

__global__ void __launch_bounds__(kTB) k_resample(int n, const double* w, const double* u0p,
                                                  const double* cond_ess, double cond_thr,
                                                  int* idx, int* degenerate,
                                                  unsigned long long* cum) {
  __shared__ ResampleLds L;
  resample_body(n, w, u0p, cond_ess, cond_thr, idx, degenerate, cum, L);
}

// dst[j][:] = src[idx[j]][:]
__global__ void k_gather(int n_rows, int64_t row_len, const int* idx, const double* src,
                         double* dst) {
  const int j = blockIdx.y;
  const int r = idx[j];
  if (r < 0 || r >= n_rows) return;  // out-of-range index: row left untouched
  const double* s = src + static_cast<int64_t>(r) * row_len;
  double* d = dst + static_cast<int64_t>(j) * row_len;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < row_len;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    d[i] = s[i];
}

// ---------------------------------------------------------------------------
// Ensemble statistics of section 4 (EMRE, RB, RES) against a truth row.
// ---------------------------------------------------------------------------
// mean[i] = (1/n) sum_p u[p][i]
__global__ void k_ens_mean(int n, int nx, const double* u, double* mean) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nx; i += gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int p = 0; p < n; ++p) acc += u[static_cast<size_t>(p) * nx + i];
    mean[i] = acc / n;
  }
}

// Per particle (one wavefront each): |ua - u_p|^2 and |u_p - mean|^2.
__global__ void __launch_bounds__(kWave) k_ens_norms(int nx, const double* u, const double* ua,
                                                     const double* mean, double* sq) {
  const int p = blockIdx.x;
  const double* up = u + static_cast<size_t>(p) * nx;
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < nx; i += kWave) {
    const double d = ua[i] - up[i], e = up[i] - mean[i];
    a = fma(d, d, a);
    b = fma(e, e, b);
  }
  a = wave_sum(a);
  b = wave_sum(b);
  if (threadIdx.x == 0) {
    sq[2 * p] = a;
    sq[2 * p + 1] = b;
  }
}

// out = (EMRE, RB, RES) from the per-particle squares (one wavefront).
__global__ void __launch_bounds__(kWave) k_ens_final(int n, int nx, const double* ua,
                                                     const double* mean, const double* sq,
                                                     double* out) {
  double na = 0.0, nb = 0.0, se = 0.0, ss = 0.0;
  for (int i = threadIdx.x; i < nx; i += kWave) {
    const double d = ua[i] - mean[i];
    na = fma(ua[i], ua[i], na);
    nb = fma(d, d, nb);
  }
  for (int p = threadIdx.x; p < n; p += kWave) {
    se += sqrt(sq[2 * p]);
    ss += sqrt(sq[2 * p + 1]);
  }
  na = wave_sum(na);
  nb = wave_sum(nb);
  se = wave_sum(se);
  ss = wave_sum(ss);
  if (threadIdx.x == 0) {
    const double nrm = sqrt(na);
    out[0] = se / n / nrm;
    out[1] = sqrt(nb) / nrm;
    out[2] = n > 1 ? ss / (n - 1) / nrm : 0.0;
  }
}

// A particle whose window failed (status != SCH_OK) gets phi = +inf: zero
// weight, so the next resampling replaces it.
__global__ void k_mask_failed(int n, const int* status, double* phi) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && status[i] != SCH_OK) phi[i] = INFINITY;
}

__global__ void k_fill(double* p, double v, int64_t n) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    p[i] = v;
}

// *out += sum of a[0 .. n) (one workgroup of 256 threads).
__global__ void __launch_bounds__(256) k_sum_i32_u64(int n, const int* a,
                                                     unsigned long long* out) {
  __shared__ unsigned long long part[256];
  unsigned long long s = 0;
  for (int i = threadIdx.x; i < n; i += 256) s += static_cast<unsigned long long>(a[i]);
  part[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (static_cast<int>(threadIdx.x) < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out += part[0];
}

__global__ void k_zero_u64(unsigned long long* p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0ull;
}

}  // namespace sch
