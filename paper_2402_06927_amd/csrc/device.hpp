// device.hpp -- device building blocks for the gfx950 SCH particle-filter
// kernels: the counter-based generator, wavefront/workgroup reductions, and
// the workgroup-wide solver for periodic (cyclic) tridiagonal systems.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sch.h"

namespace sch {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): per round, the words at
// positions 0 and 2 are multiplied by two fixed odd constants; the new word 0
// is hi(M1*c2) ^ c1 ^ k0, word 1 is lo(M1*c2), word 2 is hi(M0*c0) ^ c3 ^ k1,
// word 3 is lo(M0*c0); the 2x32-bit key advances by a Weyl increment after
// each round.
// ---------------------------------------------------------------------------
struct Ctr4 {
  uint32_t w[4];
};

__device__ __forceinline__ Ctr4 philox10(Ctr4 c, uint64_t seed) {
  constexpr uint32_t kMulA = 0xD2511F53u, kMulB = 0xCD9E8D57u;
  constexpr uint32_t kWeylA = 0x9E3779B9u, kWeylB = 0xBB67AE85u;
  uint32_t ka = static_cast<uint32_t>(seed), kb = static_cast<uint32_t>(seed >> 32);
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t hiA = __umulhi(kMulA, c.w[0]), loA = kMulA * c.w[0];
    const uint32_t hiB = __umulhi(kMulB, c.w[2]), loB = kMulB * c.w[2];
    Ctr4 n;
    n.w[0] = hiB ^ c.w[1] ^ ka;
    n.w[1] = loB;
    n.w[2] = hiA ^ c.w[3] ^ kb;
    n.w[3] = loA;
    c = n;
    ka += kWeylA;
    kb += kWeylB;
  }
  return c;
}

// 53 high bits of (hi:lo) as an exact double in [0, 1).
__device__ __forceinline__ double unit_double(uint32_t hi, uint32_t lo) {
  const uint64_t bits = (static_cast<uint64_t>(hi) << 32) | lo;
  return static_cast<double>(bits >> 11) * 0x1.0p-53;
}

// Two standard normals from one Philox block (Box-Muller on 1 - u1 in (0,1]).
__device__ __forceinline__ void normal2(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2,
                                        uint32_t c3, double& z0, double& z1) {
  const Ctr4 r = philox10(Ctr4{{c0, c1, c2, c3}}, seed);
  const double u1 = unit_double(r.w[0], r.w[1]);
  const double u2 = unit_double(r.w[2], r.w[3]);
  const double rad = sqrt(-2.0 * log(1.0 - u1));
  const double ang = 6.283185307179586 * u2;
  double sn, cs;
  sincos(ang, &sn, &cs);
  z0 = rad * cs;
  z1 = rad * sn;
}

__device__ __forceinline__ double uniform1(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2,
                                           uint32_t c3) {
  const Ctr4 r = philox10(Ctr4{{c0, c1, c2, c3}}, seed);
  return unit_double(r.w[0], r.w[1]);
}

// ---------------------------------------------------------------------------
// Cross-lane moves without LDS: DPP row shifts (a lane reads lane l -/+ d of
// its 16-lane row, or keeps `old` where no such lane exists), whole-wave
// shifts by one, and readlane broadcasts into scalar registers.
// ---------------------------------------------------------------------------
constexpr int kDppRowShr = 0x110, kDppRowShl = 0x100, kDppWaveShr1 = 0x138,
              kDppWaveShl1 = 0x130;

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double src, double old) {
  const int lo = __builtin_amdgcn_update_dpp(__double2loint(old), __double2loint(src), CTRL, 0xf,
                                             0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(__double2hiint(old), __double2hiint(src), CTRL, 0xf,
                                             0xf, false);
  return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ int dpp_i32(int src, int old) {
  return __builtin_amdgcn_update_dpp(old, src, CTRL, 0xf, 0xf, false);
}
// The same with bound control: lanes without a source lane read 0.
template <int CTRL>
__device__ __forceinline__ double dpp_f64z(double src) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(src), CTRL, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(src), CTRL, 0xf, 0xf, true);
  return __hiloint2double(hi, lo);
}
// lane must be wave-uniform
__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// ---------------------------------------------------------------------------
// Wave reductions (every lane receives the result): inclusive prefix within
// each row by row shifts, then the four row results from lanes 15, 31, 47, 63.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_f64<kDppRowShr + 1>(v, 0.0);
  v += dpp_f64<kDppRowShr + 2>(v, 0.0);
  v += dpp_f64<kDppRowShr + 4>(v, 0.0);
  v += dpp_f64<kDppRowShr + 8>(v, 0.0);
  return (readlane_f64(v, 15) + readlane_f64(v, 31)) + (readlane_f64(v, 47) + readlane_f64(v, 63));
}
__device__ __forceinline__ double wave_max(double v) {
  v = fmax(v, dpp_f64<kDppRowShr + 1>(v, v));
  v = fmax(v, dpp_f64<kDppRowShr + 2>(v, v));
  v = fmax(v, dpp_f64<kDppRowShr + 4>(v, v));
  v = fmax(v, dpp_f64<kDppRowShr + 8>(v, v));
  return fmax(fmax(readlane_f64(v, 15), readlane_f64(v, 31)),
              fmax(readlane_f64(v, 47), readlane_f64(v, 63)));
}
__device__ __forceinline__ int wave_or(int v) {
  v |= dpp_i32<kDppRowShr + 1>(v, 0);
  v |= dpp_i32<kDppRowShr + 2>(v, 0);
  v |= dpp_i32<kDppRowShr + 4>(v, 0);
  v |= dpp_i32<kDppRowShr + 8>(v, 0);
  return __builtin_amdgcn_readlane(v, 15) | __builtin_amdgcn_readlane(v, 31) |
         __builtin_amdgcn_readlane(v, 47) | __builtin_amdgcn_readlane(v, 63);
}

// ---------------------------------------------------------------------------
// Shared memory of the row solver for a workgroup of NT threads (NT a power
// of two, >= 64).
// ---------------------------------------------------------------------------
template <int NT>
struct RowLds {
  double tail_y[NT], tail_g[NT], tail_k[NT];  // last-row spike values per chunk
  double pcr[2][4][NT];                       // cyclic reduction, double buffered
  double s[NT];                               // interface unknowns
  double first[2][NT], last[2][NT];           // halo exchange, double buffered
  double red[3][NT / kWave];                  // workgroup reductions
  double helm[2][NT / kWave][8];              // per-wavefront records of solve_helm()
  int stop[16];                               // per-level "coupling remains" flags
};

// 1/x for the solvers' pivots: the hardware estimate (relative error about
// 5e-8 on gfx950) and one Newton step, which squares that error (at most
// about 11 ulp, 2e-15 relative); the pivots are bounded away from zero.
__device__ __forceinline__ double rcp64(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  return fma(r, fma(-x, r, 1.0), r);
}

// A row of the periodic mesh is split over the NT threads of a workgroup:
// thread t owns the `cnt` consecutive rows starting at `start`, held in
// register slots 0..cnt-1 (PMAX slots in total).  FULL means cnt == PMAX for
// every thread.
struct Chunk {
  int start, cnt;
};

template <int NT>
__device__ __forceinline__ Chunk chunk_of(int nx, int t) {
  const int base = nx / NT, rem = nx % NT;
  Chunk c;
  c.cnt = base + (t < rem ? 1 : 0);
  c.start = t * base + (t < rem ? t : rem);
  return c;
}

// Value of slot j's left / right neighbour given the halo values.
template <int PMAX, bool FULL>
__device__ __forceinline__ double left_of(const double (&v)[PMAX], int j, double hl) {
  return j == 0 ? hl : v[j > 0 ? j - 1 : 0];
}
template <int PMAX, bool FULL>
__device__ __forceinline__ double right_of(const double (&v)[PMAX], int j, int cnt, double hr) {
  const bool last = FULL ? (j == PMAX - 1) : (j == cnt - 1);
  return last ? hr : v[j + 1 < PMAX ? j + 1 : PMAX - 1];
}

// Publishes each thread's first and last row value and returns the left and
// right neighbours of the chunk (periodic).  The two buffers alternate
// between calls (hs toggles), so one barrier per exchange suffices: a buffer
// is rewritten only after the barrier of the exchange in between.
template <int PMAX, int NT, bool FULL>
__device__ __forceinline__ void halo(const double (&v)[PMAX], int cnt, RowLds<NT>& L, int t,
                                     double& hl, double& hr, int& hs) {
  double lastv = v[PMAX - 1];
  if (!FULL) {
    lastv = v[0];
#pragma unroll
    for (int j = 1; j < PMAX; ++j)
      if (j == cnt - 1) lastv = v[j];
  }
  L.first[hs][t] = v[0];
  L.last[hs][t] = lastv;
  __syncthreads();
  hl = L.last[hs][(t + NT - 1) & (NT - 1)];
  hr = L.first[hs][(t + 1) & (NT - 1)];
  hs ^= 1;
}

// Parallel cyclic reduction of the periodic tridiagonal system with one
// equation per thread, A_t s_{t-1} + B_t s_t + C_t s_{t+1} = R_t.  After
// log2(NT) levels every equation couples s_t only to itself.  The reduction
// stops earlier once every remaining coupling is below 2^-60 of its
// diagonal (then s_t = R_t / B_t to within rounding); the decision is shared
// through a per-level LDS flag read after the level's barrier.
template <int NT>
__device__ __forceinline__ double pcr_cyclic(double A, double B, double C, double R,
                                             RowLds<NT>& L, int t) {
  if (t < 16) L.stop[t] = 0;
  int cur = 0;
  L.pcr[0][0][t] = A;
  L.pcr[0][1][t] = B;
  L.pcr[0][2][t] = C;
  L.pcr[0][3][t] = R;
  __syncthreads();
  int level = 0;
  for (int d = 1; d < NT; d <<= 1, ++level) {
    const int tm = (t - d) & (NT - 1), tp = (t + d) & (NT - 1);
    const double Am = L.pcr[cur][0][tm], Bm = L.pcr[cur][1][tm], Cm = L.pcr[cur][2][tm],
                 Rm = L.pcr[cur][3][tm];
    const double Ap = L.pcr[cur][0][tp], Bp = L.pcr[cur][1][tp], Cp = L.pcr[cur][2][tp],
                 Rp = L.pcr[cur][3][tp];
    const double k1 = A * rcp64(Bm), k2 = C * rcp64(Bp);
    const double nA = -k1 * Am;
    const double nB = B - k1 * Cm - k2 * Ap;
    const double nC = -k2 * Cp;
    const double nR = R - k1 * Rm - k2 * Rp;
    A = nA;
    B = nB;
    C = nC;
    R = nR;
    cur ^= 1;
    L.pcr[cur][0][t] = A;
    L.pcr[cur][1][t] = B;
    L.pcr[cur][2][t] = C;
    L.pcr[cur][3][t] = R;
    if (__any(fabs(A) + fabs(C) > 0x1.0p-60 * fabs(B)) && (t & (kWave - 1)) == 0)
      atomicOr(&L.stop[level], 1);
    __syncthreads();
    if (L.stop[level] == 0) return R * rcp64(B);
  }
  return R * rcp64(A + B + C);
}

// Workgroup solve of the periodic tridiagonal system
//     a_i x_{i-1} + b_i x_i + c_i x_{i+1} = d_i   (indices mod nx)
// distributed as chunks of rows per thread.  Partition method: the first row
// of every chunk is an interface unknown s_t; each thread eliminates its
// remaining rows by Thomas' algorithm into x_j = y_j + g_j s_t + k_j s_{t+1}
// (two spike columns), the interface rows form a periodic tridiagonal system
// of NT unknowns solved by cyclic reduction, and the chunk is recombined.
// row(j, a, b, c) returns the coefficients of local slot j and d(j) its
// right-hand side (both evaluated once per slot).  xl and xr receive the
// solution at the row before the chunk and the row after it (the halo of x,
// from the interface values, without another exchange).  No pivoting: the
// systems solved here (mass, Helmholtz and the implicit-midpoint matrix at
// the model's parameters) are diagonally dominant.
template <int PMAX, int NT, bool FULL, class RowF, class DF>
__device__ __forceinline__ void cyclic_solve(RowF row, DF d, double (&x)[PMAX], int cnt,
                                             RowLds<NT>& L, int t, double& xl, double& xr) {
  static_assert(PMAX >= 2, "need at least two rows per thread");
  double cp[PMAX], g[PMAX];
  // forward elimination over the interior slots 1..cnt-1; inactive slots
  // (j >= cnt) are given c' = -1, y' = g' = 0 so the back sweep passes the
  // right-spike seed (k = 1) and zeros through them unchanged.
  double cprev = 0.0, yprev = 0.0, gprev = 1.0;
#pragma unroll
  for (int j = 1; j < PMAX; ++j) {
    double a, b, c;
    row(j, a, b, c);
    const double inv = rcp64(b - a * cprev);
    double cj = c * inv, yj = (d(j) - a * yprev) * inv, gj = -a * gprev * inv;
    if (!FULL && j >= cnt) {
      cj = -1.0;
      yj = 0.0;
      gj = 0.0;
    }
    cp[j] = cj;
    x[j] = yj;
    g[j] = gj;
    cprev = cj;
    yprev = yj;
    gprev = gj;
  }
  // back substitution for y and both spikes; the right spike k_j is the
  // running product of -c'_i over i = j..PMAX-1 and is rebuilt when needed
  double yn = 0.0, gn = 0.0, kn = 1.0;
  double yL = 0.0, gL = 1.0, kL = 0.0;  // last row of the chunk (the interface if cnt == 1)
#pragma unroll
  for (int j = PMAX - 1; j >= 1; --j) {
    const double yj = x[j] - cp[j] * yn;
    const double gj = g[j] - cp[j] * gn;
    const double kj = -cp[j] * kn;
    x[j] = yj;
    g[j] = gj;
    yn = yj;
    gn = gj;
    kn = kj;
    if (!FULL && j == cnt - 1) {
      yL = yj;
      gL = gj;
      kL = kj;
    }
    if (FULL && j == PMAX - 1) {
      yL = yj;
      gL = gj;
      kL = kj;
    }
  }
  // interface equation of chunk t
  L.tail_y[t] = yL;
  L.tail_g[t] = gL;
  L.tail_k[t] = kL;
  __syncthreads();
  const int tm = (t + NT - 1) & (NT - 1);
  const double ypl = L.tail_y[tm], gpl = L.tail_g[tm], kpl = L.tail_k[tm];
  double a0, b0, c0;
  row(0, a0, b0, c0);
  const double A = a0 * gpl;
  const double B = b0 + a0 * kpl + c0 * gn;
  const double C = c0 * kn;
  const double R = d(0) - a0 * ypl - c0 * yn;
  const double s = pcr_cyclic<NT>(A, B, C, R, L, t);
  L.s[t] = s;
  __syncthreads();
  const double snext = L.s[(t + 1) & (NT - 1)];
  // last row of chunk t-1: y + g s_{t-1} + k s_t with its tail values
  xl = fma(kpl, s, fma(gpl, L.s[tm], ypl));
  xr = snext;
  x[0] = s;
  double kr = 1.0;
#pragma unroll
  for (int j = PMAX - 1; j >= 1; --j) {
    kr *= -cp[j];
    x[j] = x[j] + g[j] * s + kr * snext;
  }
}

// Workgroup-wide max of two values and logical or of a flag.
template <int NT>
__device__ __forceinline__ void block_max2_or(double& a, double& b, int& f, RowLds<NT>& L, int t) {
  a = wave_max(a);
  b = wave_max(b);
  f = wave_or(f);
  const int w = t / kWave;
  if ((t & (kWave - 1)) == 0) {
    L.red[0][w] = a;
    L.red[1][w] = b;
    L.red[2][w] = f ? 1.0 : 0.0;
  }
  __syncthreads();
  a = L.red[0][0];
  b = L.red[1][0];
  double ff = L.red[2][0];
#pragma unroll
  for (int i = 1; i < NT / kWave; ++i) {
    a = fmax(a, L.red[0][i]);
    b = fmax(b, L.red[1][i]);
    ff = fmax(ff, L.red[2][i]);
  }
  f = ff > 0.0;
  __syncthreads();
}

template <int NT>
__device__ __forceinline__ double block_sum(double a, RowLds<NT>& L, int t) {
  a = wave_sum(a);
  if ((t & (kWave - 1)) == 0) L.red[0][t / kWave] = a;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < NT / kWave; ++i) s += L.red[0][i];
  __syncthreads();
  return s;
}

}  // namespace sch
