// helm.hpp -- workgroup solve of the constant periodic Helmholtz system
// H u = f, H = d I + o (S + S^{-1}) (S the cyclic shift; d = 2h/3 + 2 alpha^2/h,
// o = h/6 - alpha^2/h from the first line of eq. fde1), in one barrier.
//
// H factors as kappa (1 - r S)(1 - r S^{-1}) with r the root in (0,1) of
// r^2 + (d/o) r + 1 = 0 and kappa = -o/r, so
//   H^{-1} f = (F+ + F- - f) / (kappa (1 - r^2)),
// where F+ and F- are the periodic solutions of the first-order recurrences
// F+_i = f_i + r F+_{i-1} and F-_i = f_i + r F-_{i+1}.  Both recurrences are
// linear scans: each thread scans its chunk, the chunk carries are combined
// across lanes by shuffles and across wavefronts through one LDS record per
// wavefront, and the periodic images add r^(i+1) G+_{N-1} / (1 - r^N) (resp.
// r^(N-i) G-_0 / (1 - r^N)) to the non-periodic scans G+-.  The record also
// carries three reduction partials, so a caller can fold a workgroup
// reduction into the same barrier.
#pragma once

#include "device.hpp"

namespace sch {

struct HelmConst {
  double r, coef;   // root and 1/(kappa (1 - r^2)), kappa = -o / r
  double rN1;       // 1/(1 - r^nx)
  double rb, rb1;   // r^base, r^(base+1): multipliers of chunks of base / base+1 rows
  int base;         // nx / NT
  double ho, hd;    // off-diagonal and diagonal of H
};

// Composition of affine carries: apply (m1, c1) then (m2, c2).
__device__ __forceinline__ void compose(double m1, double c1, double m2, double c2, double& m,
                                        double& c) {
  m = m1 * m2;
  c = fma(m2, c1, c2);
}

template <int PMAX, int NT, bool FULL, class LT>
__device__ __forceinline__ void solve_helm(const HelmConst& K, const double (&f)[PMAX],
                                           double (&u)[PMAX], double& uL, double& uR, int cnt,
                                           LT& L, int slot, int t, double red0, double red1,
                                           double red2, double& gred0, double& gred1,
                                           double& gred2) {
  constexpr int W = NT / kWave;
  const int lane = t & (kWave - 1), wv = t / kWave;
  const double r = K.r;
  // local scans; sc[j] = (forward + backward - f) local sums
  double sc[PMAX];
  double acc = 0.0;
#pragma unroll
  for (int j = 0; j < PMAX; ++j) {
    acc = (FULL || j < cnt) ? fma(r, acc, f[j]) : acc;
    sc[j] = acc - f[j];
  }
  const double cpl = acc;  // forward carry out of the chunk
  acc = 0.0;
#pragma unroll
  for (int j = PMAX - 1; j >= 0; --j) {
    if (FULL || j < cnt) acc = fma(r, acc, f[j]);
    sc[j] += acc;
  }
  const double cmn = acc;  // backward carry out of the chunk (at its first node)
  const double mth = (FULL || cnt == K.base) ? K.rb : K.rb1;
  // inclusive scans over lanes: forward (m, c) composes lanes 0..lane,
  // backward composes lanes lane..63
  double fm = mth, fc = cpl, bm = mth, bc = cmn;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const double pm = __shfl_up(fm, d), pc = __shfl_up(fc, d);
    const double qm = __shfl_down(bm, d), qc = __shfl_down(bc, d);
    if (lane >= d) compose(pm, pc, fm, fc, fm, fc);
    if (lane + d < kWave) compose(qm, qc, bm, bc, bm, bc);
  }
  // exclusive values within the wavefront
  double xfm = __shfl_up(fm, 1), xfc = __shfl_up(fc, 1);
  double xbm = __shfl_down(bm, 1), xbc = __shfl_down(bc, 1);
  if (lane == 0) {
    xfm = 1.0;
    xfc = 0.0;
  }
  if (lane == kWave - 1) {
    xbm = 1.0;
    xbc = 0.0;
  }
  // wavefront totals and reduction partials to LDS
  const double tfm = __shfl(fm, kWave - 1), tfc = __shfl(fc, kWave - 1);
  const double tbm = __shfl(bm, 0), tbc = __shfl(bc, 0);
  if (lane == 0) {
    double* rec = L.helm[slot][wv];
    rec[0] = tfm;
    rec[1] = tfc;
    rec[2] = tbm;
    rec[3] = tbc;
    rec[4] = red0;
    rec[5] = red1;
    rec[6] = red2;
  }
  __syncthreads();
  // Combine the W records: lane v < W of every wavefront takes record v; the
  // forward records compose left to right, the backward ones right to left,
  // by shuffle scans over those lanes (identities in the other lanes).
  double f0 = 1.0, f1 = 0.0, b0 = 1.0, b1 = 0.0, q0 = 0.0, q1 = 0.0, q2 = 0.0;
  if (lane < W) {
    const double* rec = L.helm[slot][lane];
    f0 = rec[0];
    f1 = rec[1];
    b0 = rec[2];
    b1 = rec[3];
    q0 = rec[4];
    q1 = rec[5];
    q2 = rec[6];
  }
#pragma unroll
  for (int d = 1; d < W; d <<= 1) {
    const double pm = __shfl_up(f0, d), pc = __shfl_up(f1, d);
    const double qm = __shfl_down(b0, d), qc = __shfl_down(b1, d);
    if (lane >= d) compose(pm, pc, f0, f1, f0, f1);
    if (lane + d < W) compose(qm, qc, b0, b1, b0, b1);
    q0 = fmax(q0, __shfl_xor(q0, d));
    q1 = fmax(q1, __shfl_xor(q1, d));
    q2 = fmax(q2, __shfl_xor(q2, d));
  }
  // lanes >= W reduced zeros among themselves: take lane 0's maxima
  gred0 = __shfl(q0, 0);
  gred1 = __shfl(q1, 0);
  gred2 = __shfl(q2, 0);
  // totals, and the carries entering this wavefront from the left / right
  const double allfm = __shfl(f0, W - 1), allfc = __shfl(f1, W - 1);
  const double allbm = __shfl(b0, 0), allbc = __shfl(b1, 0);
  double inm = __shfl(f0, wv > 0 ? wv - 1 : 0), inc = __shfl(f1, wv > 0 ? wv - 1 : 0);
  double rim = __shfl(b0, wv + 1 < W ? wv + 1 : 0), ric = __shfl(b1, wv + 1 < W ? wv + 1 : 0);
  if (wv == 0) {
    inm = 1.0;
    inc = 0.0;
  }
  if (wv == W - 1) {
    rim = 1.0;
    ric = 0.0;
  }
  (void)allfm;
  (void)allbm;
  // thread-exclusive carries: forward carry at node start-1, product r^start;
  // backward carry at node end+1, product r^(nx - end - 1)
  double pfm, pfc, pbm, pbc;
  compose(inm, inc, xfm, xfc, pfm, pfc);
  compose(rim, ric, xbm, xbc, pbm, pbc);
  // periodic images: Gamma+ = G+_{N-1} / (1 - r^N), Gamma- = G-_0 / (1 - r^N)
  const double gamp = allfc * K.rN1, gamm = allbc * K.rN1;
  const double Ep = fma(pfm, gamp, pfc);
  const double Em = fma(pbm, gamm, pbc);
  // u_j = coef (sc_j + r^(j+1) Ep + r^(cnt-j) Em): the backward factor is
  // r^(cnt-j) = r^cnt / r^j, built from the chunk multiplier; the forward
  // factor grows by r per slot
  double rf = r;
  double rbk = mth;  // r^(cnt - j), starting at j = 0
  const double ir = 1.0 / r;
#pragma unroll
  for (int j = 0; j < PMAX; ++j) {
    u[j] = K.coef * fma(rbk, Em, fma(rf, Ep, sc[j]));
    rf *= r;
    rbk *= ir;
  }
  // bordering values from the Helmholtz rows of the first and last node,
  // o u_{i-1} + d u_i + o u_{i+1} = f_i (meaningful for chunks of >= 2 rows)
  const int last = FULL ? PMAX - 1 : cnt - 1;
  double ul = u[PMAX - 1], ulm = u[PMAX - 2], fl = f[PMAX - 1];
  if (!FULL) {
#pragma unroll
    for (int j = 1; j < PMAX; ++j)
      if (j == last) {
        ul = u[j];
        ulm = u[j - 1];
        fl = f[j];
      }
  }
  const double iho = 1.0 / K.ho;
  uL = (f[0] - K.hd * u[0] - K.ho * u[1]) * iho;
  uR = (fl - K.hd * ul - K.ho * ulm) * iho;
}

}  // namespace sch
