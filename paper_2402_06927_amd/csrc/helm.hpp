// helm.hpp -- workgroup solve of the constant periodic Helmholtz system
// H u = f (or H u = M f), H = d I + o (S + S^{-1}) (S the cyclic shift; d = 2h/3 + 2 alpha^2/h,
// o = h/6 - alpha^2/h from the first line of eq. fde1), in one barrier.
//
// H factors as kappa (1 - r S)(1 - r S^{-1}) with r the root of modulus < 1 of
// r^2 + (d/o) r + 1 = 0 and kappa = -o/r, so
//   H^{-1} f = (F+ + F- - f) / (kappa (1 - r^2)),
// where F+ and F- are the periodic solutions of the first-order recurrences
// F+_i = f_i + r F+_{i-1} and F-_i = f_i + r F-_{i+1}.  Both recurrences are
// linear scans: each thread scans its chunk, the chunk carries are combined
// across lanes by DPP row shifts and readlane and across wavefronts through
// one LDS record per wavefront, and the periodic images add r^(i+1) G+_{N-1} / (1 - r^N) (resp.
// r^(N-i) G-_0 / (1 - r^N)) to the non-periodic scans G+-.  The record also
// carries three nonnegative reduction partials, so a caller can fold a
// workgroup max-reduction into the same barrier; the first comes back as
// +infinity when the right-hand side holds a non-finite value.
#pragma once

#include "device.hpp"

namespace sch {

struct HelmConst {
  double r, coef;   // root and 1/(kappa (1 - r^2)), kappa = -o / r
  double rinv;      // 1 / r
  double rN1;       // 1/(1 - r^nx)
  double rb, rb1;   // r^base, r^(base+1): multipliers of chunks of base / base+1 rows
  int base;         // nx / NT
  double ho, hd;    // off-diagonal and diagonal of H
  // The mass matrix M (rows h/6, 2h/3, h/6) lies in the span of I and H:
  // M = beta H + gamma I with beta = (h/6) / ho, gamma = 2h/3 - beta hd, so
  // H^{-1} M f = beta f + gamma H^{-1} f = mg (F+ + F-) + mf f with
  // mg = gamma coef and mf = beta - gamma coef (the scan form below).
  double mg, mf;
  double mh6, mh23;  // h/6 and 2h/3
  // rb^e for e = 0..64, formed on the host by the same binary powering as
  // the solve's own (the products rb^(2^i) in increasing i): the PWT solves
  // read the lane scans' factors from this table
  double pwt[65];
};

// Composition of affine carries: apply (m1, c1) then (m2, c2).
__device__ __forceinline__ void compose(double m1, double c1, double m2, double c2, double& m,
                                        double& c) {
  m = m1 * m2;
  c = fma(m2, c1, c2);
}

// Inclusive affine scan inside each 16-lane row: CTRL = row shift right
// (forward: compose the lanes to the left first) or left (backward: the
// lanes to the right first).
template <int CTRL>
__device__ __forceinline__ void scan_rows(double& m, double& c) {
#pragma unroll
  for (int d = 1; d < 16; d <<= 1) {
    double pm, pc;
    if (d == 1) { pm = dpp_f64<CTRL + 1>(m, 1.0); pc = dpp_f64z<CTRL + 1>(c); }
    else if (d == 2) { pm = dpp_f64<CTRL + 2>(m, 1.0); pc = dpp_f64z<CTRL + 2>(c); }
    else if (d == 4) { pm = dpp_f64<CTRL + 4>(m, 1.0); pc = dpp_f64z<CTRL + 4>(c); }
    else { pm = dpp_f64<CTRL + 8>(m, 1.0); pc = dpp_f64z<CTRL + 8>(c); }
    compose(pm, pc, m, c, m, c);
  }
}

// Scans of the per-wavefront records held in lanes 0..W-1 (W <= 8): forward
// and backward affine compositions and running maxima of three nonnegative
// partials (lanes without a partner contribute the identities 1, 0 and 0).
template <int W>
__device__ __forceinline__ void record_scan(double& f0, double& f1, double& b0, double& b1,
                                            double& q0, double& q1, double& q2) {
#define SCH_RSTEP(D)                                                              \
  if constexpr (W > D) {                                                          \
    double pm = dpp_f64<kDppRowShr + D>(f0, 1.0), pc = dpp_f64z<kDppRowShr + D>(f1); \
    compose(pm, pc, f0, f1, f0, f1);                                              \
    double qm = dpp_f64<kDppRowShl + D>(b0, 1.0), qc = dpp_f64z<kDppRowShl + D>(b1); \
    compose(qm, qc, b0, b1, b0, b1);                                              \
    q0 = vmax(q0, dpp_f64z<kDppRowShr + D>(q0));                                  \
    q1 = vmax(q1, dpp_f64z<kDppRowShr + D>(q1));                                  \
    q2 = vmax(q2, dpp_f64z<kDppRowShr + D>(q2));                                  \
  }
  SCH_RSTEP(1)
  SCH_RSTEP(2)
  SCH_RSTEP(4)
#undef SCH_RSTEP
}

// MASS: u = H^{-1} M f instead of H^{-1} f, with fl, fr the values of f at
// the nodes bordering the chunk (for the bordering values of u).
// PWT (full chunks): the lane scans' powers of r^PMAX are loaded from K.pwt
// at every call instead of being formed per lane.  Formed powers are loop
// invariants that the compiler hoists out of the caller's loops into
// registers; where registers are short (the kernels with the Matern-type
// noise, which also hold that operator's powers) they are spilled and
// reloaded from scratch every iteration, and loading them from the table
// is cheaper.  Elsewhere forming them costs fewer instructions.  Both give
// the same bits.
template <int PMAX, int NT, bool FULL, bool MASS = false, bool PWT = false, class LT>
__device__ __forceinline__ void solve_helm(const HelmConst& K, const double (&f)[PMAX],
                                           double (&u)[PMAX], double& uL, double& uR, int cnt,
                                           LT& L, int slot, int t, double red0, double red1,
                                           double red2, double& gred0, double& gred1,
                                           double& gred2, double fl = 0.0, double fr = 0.0) {
  constexpr int W = NT / kWave;
  const int lane = t & (kWave - 1), wv = t / kWave;
  const double r = K.r;
  // carries out of the chunk: the local forward scan at its last node and
  // the local backward scan at its first node
  double acc = 0.0;
#pragma unroll
  for (int j = 0; j < PMAX; ++j) acc = slot_live<PMAX, FULL>(j, cnt) ? fma(r, acc, f[j]) : acc;
  const double cpl = acc;
  acc = 0.0;
#pragma unroll
  for (int j = PMAX - 1; j >= 0; --j) acc = slot_live<PMAX, FULL>(j, cnt) ? fma(r, acc, f[j]) : acc;
  const double cmn = acc;
  const double mth = (FULL || cnt == K.base) ? K.rb : K.rb1;
  const int row = lane >> 4;
  double fc = cpl, bc = cmn;          // offsets of the inclusive scans
  double xfm, xfc, xbm, xbc;          // exclusive carries within the wavefront
  double tfm, tfc, tbm, tbc;          // wavefront totals
  if constexpr (FULL) {
    // Every chunk has PMAX rows, so the factor of any run of lanes is a
    // power of r^PMAX: only the offsets need cross-lane steps.
    const double* pt = K.pwt;
    int ln = lane;
    if constexpr (PWT) {
      // opaque indices keep the loads at the call (scalar loads for the
      // uniform powers, four vector loads of the table for the per-lane ones)
      int z = 0;
      asm volatile("" : "+s"(z));
      pt += z;
      asm volatile("" : "+v"(ln));
    }
    const double rb = PWT ? pt[1] : K.rb, rb2 = PWT ? pt[2] : rb * rb,
                 rb4 = PWT ? pt[4] : rb2 * rb2, rb8 = PWT ? pt[8] : rb4 * rb4,
                 rb16 = PWT ? pt[16] : rb8 * rb8, rb32 = rb16 * rb16,
                 rb64 = PWT ? pt[64] : rb32 * rb32;
    auto pw = [&](int e) {  // rb^e, 0 <= e <= 64
      if constexpr (PWT) return pt[e];
      double p = (e & 1) ? rb : 1.0;
      p *= (e & 2) ? rb2 : 1.0;
      p *= (e & 4) ? rb4 : 1.0;
      p *= (e & 8) ? rb8 : 1.0;
      p *= (e & 16) ? rb16 : 1.0;
      p *= (e & 32) ? rb32 : 1.0;
      return (e & 64) ? p * rb64 : p;
    };
    const int i16 = ln & 15;
    fc = fma(rb, dpp_f64z<kDppRowShr + 1>(fc), fc);
    fc = fma(rb2, dpp_f64z<kDppRowShr + 2>(fc), fc);
    fc = fma(rb4, dpp_f64z<kDppRowShr + 4>(fc), fc);
    fc = fma(rb8, dpp_f64z<kDppRowShr + 8>(fc), fc);
    bc = fma(rb, dpp_f64z<kDppRowShl + 1>(bc), bc);
    bc = fma(rb2, dpp_f64z<kDppRowShl + 2>(bc), bc);
    bc = fma(rb4, dpp_f64z<kDppRowShl + 4>(bc), bc);
    bc = fma(rb8, dpp_f64z<kDppRowShl + 8>(bc), bc);
    {
      const double r0c = readlane_f64(fc, 15), r1c = readlane_f64(fc, 31),
                   r2c = readlane_f64(fc, 47);
      const double p2c = fma(rb16, r0c, r1c), p3c = fma(rb16, p2c, r2c);
      const double pc = row == 0 ? 0.0 : row == 1 ? r0c : row == 2 ? p2c : p3c;
      fc = fma(pw(i16 + 1), pc, fc);
      const double t1c = readlane_f64(bc, 16), t2c = readlane_f64(bc, 32),
                   t3c = readlane_f64(bc, 48);
      const double h1c = fma(rb16, t3c, t2c), h0c = fma(rb16, h1c, t1c);
      const double hc = row == 3 ? 0.0 : row == 2 ? t3c : row == 1 ? h1c : h0c;
      bc = fma(pw(16 - i16), hc, bc);
    }
    xfm = pw(ln);
    xfc = dpp_f64z<kDppWaveShr1>(fc);
    xbm = pw(kWave - 1 - ln);
    xbc = dpp_f64z<kDppWaveShl1>(bc);
    tfm = rb64;
    tfc = readlane_f64(fc, kWave - 1);
    tbm = rb64;
    tbc = readlane_f64(bc, 0);
  } else {
    // Inclusive scans over the lanes, forward (lanes 0..lane) and backward
    // (lanes lane..63): Hillis-Steele steps inside each 16-lane row by DPP
    // row shifts (identity where the row has no partner), then the rows are
    // joined with the row results read from the row ends into scalar
    // registers.
    double fm = mth, bm = mth;
    scan_rows<kDppRowShr>(fm, fc);
    scan_rows<kDppRowShl>(bm, bc);
    {
      const double r0m = readlane_f64(fm, 15), r0c = readlane_f64(fc, 15);
      const double r1m = readlane_f64(fm, 31), r1c = readlane_f64(fc, 31);
      const double r2m = readlane_f64(fm, 47), r2c = readlane_f64(fc, 47);
      double p2m, p2c, p3m, p3c;
      compose(r0m, r0c, r1m, r1c, p2m, p2c);
      compose(p2m, p2c, r2m, r2c, p3m, p3c);
      const double pm = row == 0 ? 1.0 : row == 1 ? r0m : row == 2 ? p2m : p3m;
      const double pc = row == 0 ? 0.0 : row == 1 ? r0c : row == 2 ? p2c : p3c;
      compose(pm, pc, fm, fc, fm, fc);
      const double t1m = readlane_f64(bm, 16), t1c = readlane_f64(bc, 16);
      const double t2m = readlane_f64(bm, 32), t2c = readlane_f64(bc, 32);
      const double t3m = readlane_f64(bm, 48), t3c = readlane_f64(bc, 48);
      double h1m, h1c, h0m, h0c;
      compose(t3m, t3c, t2m, t2c, h1m, h1c);
      compose(h1m, h1c, t1m, t1c, h0m, h0c);
      const double hm = row == 3 ? 1.0 : row == 2 ? t3m : row == 1 ? h1m : h0m;
      const double hc = row == 3 ? 0.0 : row == 2 ? t3c : row == 1 ? h1c : h0c;
      compose(hm, hc, bm, bc, bm, bc);
    }
    // exclusive values within the wavefront (identity at the ends)
    xfm = dpp_f64<kDppWaveShr1>(fm, 1.0);
    xfc = dpp_f64z<kDppWaveShr1>(fc);
    xbm = dpp_f64<kDppWaveShl1>(bm, 1.0);
    xbc = dpp_f64z<kDppWaveShl1>(bc);
    tfm = readlane_f64(fm, kWave - 1);
    tfc = readlane_f64(fc, kWave - 1);
    tbm = readlane_f64(bm, 0);
    tbc = readlane_f64(bc, 0);
  }
  // wavefront totals and reduction partials to LDS
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
  // Combine the W records: lane v < W of every wavefront takes record v
  // (identities elsewhere); forward records compose left to right, backward
  // ones right to left, by DPP steps inside row 0; the values this wavefront
  // needs are read back with readlane.
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
  record_scan<W>(f0, f1, b0, b1, q0, q1, q2);
  gred0 = readlane_f64(q0, W - 1);
  gred1 = readlane_f64(q1, W - 1);
  gred2 = readlane_f64(q2, W - 1);
  const double allfc = readlane_f64(f1, W - 1);
  // the row's forward total is finite iff every f_j is: a non-finite input
  // reports gred0 = +infinity
  if (!(fabs(allfc) <= 1.7976931348623157e308)) gred0 = INFINITY;
  const double allbc = readlane_f64(b1, 0);
  const int wvu = __builtin_amdgcn_readfirstlane(wv);
  double inm = 1.0, inc = 0.0, rim = 1.0, ric = 0.0;
  if (wvu > 0) {
    inm = readlane_f64(f0, wvu - 1);
    inc = readlane_f64(f1, wvu - 1);
  }
  if (wvu + 1 < W) {
    rim = readlane_f64(b0, wvu + 1);
    ric = readlane_f64(b1, wvu + 1);
  }
  // thread-exclusive carries: forward carry at node start-1, product r^start;
  // backward carry at node end+1, product r^(nx - end - 1)
  double pfm, pfc, pbm, pbc;
  compose(inm, inc, xfm, xfc, pfm, pfc);
  compose(rim, ric, xbm, xbc, pbm, pbc);
  // periodic images: Gamma+ = G+_{N-1} / (1 - r^N), Gamma- = G-_0 / (1 - r^N)
  const double gamp = allfc * K.rN1, gamm = allbc * K.rN1;
  const double Ep = fma(pfm, gamp, pfc);
  const double Em = fma(pbm, gamm, pbc);
  // the global scans inside the chunk, rerun from the carries into it:
  // F+_j = f_j + r F+_{j-1} from F+_{start-1} = Ep, F-_j = f_j + r F-_{j+1}
  // from F-_{end+1} = Em; u_j = coef (F+_j + F-_j - f_j)
  acc = Ep;
#pragma unroll
  for (int j = 0; j < PMAX; ++j) {
    acc = slot_live<PMAX, FULL>(j, cnt) ? fma(r, acc, f[j]) : acc;
    u[j] = MASS ? acc : acc - f[j];
  }
  acc = Em;
#pragma unroll
  for (int j = PMAX - 1; j >= 0; --j) {
    acc = slot_live<PMAX, FULL>(j, cnt) ? fma(r, acc, f[j]) : acc;
    u[j] = MASS ? fma(K.mg, u[j] + acc, K.mf * f[j]) : K.coef * (u[j] + acc);
  }
  // bordering values from the Helmholtz rows of the first and last node,
  // o u_{i-1} + d u_i + o u_{i+1} = g_i with g = f, or g = M f (MASS)
  // (meaningful for chunks of >= 2 rows)
  const int last = FULL ? PMAX - 1 : cnt - 1;
  double ul = u[PMAX - 1], ulm = u[PMAX - 2], fla = f[PMAX - 1], flm = f[PMAX - 2];
  if (!FULL) {
#pragma unroll
    for (int j = 1; j < PMAX; ++j)
      if (j >= kMinRows<PMAX> - 1 && j == last) {
        ul = u[j];
        ulm = u[j - 1];
        fla = f[j];
        flm = f[j - 1];
      }
  }
  const double g0 = MASS ? fma(K.mh6, fl + f[1], K.mh23 * f[0]) : f[0];
  const double gl = MASS ? fma(K.mh6, flm + fr, K.mh23 * fla) : fla;
  const double iho = 1.0 / K.ho;
  uL = (g0 - K.hd * u[0] - K.ho * u[1]) * iho;
  uR = (gl - K.hd * ul - K.ho * ulm) * iho;
}

}  // namespace sch
