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
// The same with bound control: lanes without a source lane read 0 (no old
// value, so no register copy ahead of the move).
template <int CTRL>
__device__ __forceinline__ double dpp_f64z(double src) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(src), CTRL, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(src), CTRL, 0xf, 0xf, true);
  return __hiloint2double(hi, lo);
}
// Row broadcast into the rows selected by ROWS; the other rows' results are
// undefined (callers read only lanes of the selected rows afterwards).
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_f64b(double src) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(src), CTRL, ROWS, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(src), CTRL, ROWS, 0xf, false);
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
  v += dpp_f64z<kDppRowShr + 1>(v);
  v += dpp_f64z<kDppRowShr + 2>(v);
  v += dpp_f64z<kDppRowShr + 4>(v);
  v += dpp_f64z<kDppRowShr + 8>(v);
  return (readlane_f64(v, 15) + readlane_f64(v, 31)) + (readlane_f64(v, 47) + readlane_f64(v, 63));
}
// max of two doubles as one v_max_f64: fmax() would first canonicalise
// operands that arrive through lane moves (two more instructions each); the
// operands here are results of arithmetic, never signalling NaNs.
__device__ __forceinline__ double vmax(double a, double b) {
  double r;
  asm("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
// max(acc, |x|) as one v_max_f64 with the absolute-value source modifier (for
// accumulating the growth of an elimination; a NaN x leaves acc unchanged).
__device__ __forceinline__ double vmax_abs(double acc, double x) {
  double r;
  asm("v_max_f64 %0, %1, |%2|" : "=v"(r) : "v"(acc), "v"(x));
  return r;
}
// (of nonnegative values: lanes without a partner take 0).  After the row
// steps, lane 15 of each row is broadcast into the next row and lane 31 into
// rows 2 and 3, so lane 63 holds the wave's maximum.
constexpr int kDppRowBcast15 = 0x142, kDppRowBcast31 = 0x143;
__device__ __forceinline__ double wave_max(double v) {
  v = vmax(v, dpp_f64z<kDppRowShr + 1>(v));
  v = vmax(v, dpp_f64z<kDppRowShr + 2>(v));
  v = vmax(v, dpp_f64z<kDppRowShr + 4>(v));
  v = vmax(v, dpp_f64z<kDppRowShr + 8>(v));
  v = vmax(v, dpp_f64b<kDppRowBcast15, 0xa>(v));
  v = vmax(v, dpp_f64b<kDppRowBcast31, 0xc>(v));
  return readlane_f64(v, 63);
}
// An upper bound, within a relative 2^-20, of the wave's maximum of
// nonnegative doubles: the maximum of the high words, each raised by one
// unit where the low word is not zero.  The 32-bit maximum fuses with the
// lane moves (one instruction per row step instead of three).
__device__ __forceinline__ double wave_max_bound(double v) {
  uint32_t h = static_cast<uint32_t>(__double2hiint(v)) + (__double2loint(v) != 0 ? 1u : 0u);
  h = max(h, static_cast<uint32_t>(__builtin_amdgcn_mov_dpp(static_cast<int>(h), kDppRowShr + 1,
                                                            0xf, 0xf, true)));
  h = max(h, static_cast<uint32_t>(__builtin_amdgcn_mov_dpp(static_cast<int>(h), kDppRowShr + 2,
                                                            0xf, 0xf, true)));
  h = max(h, static_cast<uint32_t>(__builtin_amdgcn_mov_dpp(static_cast<int>(h), kDppRowShr + 4,
                                                            0xf, 0xf, true)));
  h = max(h, static_cast<uint32_t>(__builtin_amdgcn_mov_dpp(static_cast<int>(h), kDppRowShr + 8,
                                                            0xf, 0xf, true)));
  const uint32_t m = max(max(static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(h), 15)),
                             static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(h), 31))),
                         max(static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(h), 47)),
                             static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(h), 63))));
  return __hiloint2double(static_cast<int>(m), 0);
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
// of two, 64..512).  Values cross lanes of one wavefront by DPP and
// ds_bpermute; only what crosses wavefronts goes through LDS.
// ---------------------------------------------------------------------------
template <int NT>
struct RowLds {
  static constexpr int W = NT / kWave;
  // interface equations (A, B, C, R), one per chunk, equation t at
  // eq_pos(t) = (t % W) * 65 + t / W: a lane's W consecutive equations lie
  // 65 words apart, so both the writes (one per thread) and the reads (W per
  // lane) touch consecutive banks
  double eq[4][65 * W];
  double etail[3][W];          // last-row spike values of each wavefront's last chunk
  double edge[2][W][6];        // wavefront edge values of halo exchanges, double buffered
  double red[3][W];            // workgroup reductions
  double helm[2][W][8];        // per-wavefront records of solve_helm()
};

template <int NT>
__device__ __forceinline__ int eq_pos(int t) {
  constexpr int W = NT / kWave;
  return (t % W) * 65 + t / W;
}

// 1/x for the solvers' pivots: the hardware estimate (relative error about
// 5e-8 on gfx950) and one Newton step, which squares that error (at most
// about 11 ulp, 2e-15 relative).  Small pivots are not excluded by the
// matrices themselves: an elimination that meets them grows its eliminated
// super-diagonal, which the solvers measure (kMaxGrowth below).
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

// Rows every chunk holds: chunk_of deals nx / NT or nx / NT + 1 rows, and the
// tiles (tile_for) take 8 slots only when nx > 4 NT, 16 only when nx > 8 NT,
// and always nx >= NT; the host refuses a tile that breaks this.  Slots below
// kMinRows are live in every chunk, so the masks of ragged chunks start there
// (compile-time true below it).
template <int PMAX>
inline constexpr int kMinRows = PMAX >= 8 ? PMAX / 2 : 1;
template <int PMAX, bool FULL>
__device__ __forceinline__ bool slot_live(int j, int cnt) {
  return FULL || j < kMinRows<PMAX> || j < cnt;
}
// slot j is the chunk's last live one
template <int PMAX, bool FULL>
__device__ __forceinline__ bool slot_last(int j, int cnt) {
  return FULL ? j == PMAX - 1 : (j >= kMinRows<PMAX> - 1 && j == cnt - 1);
}

// Value of slot j's left / right neighbour given the halo values.
template <int PMAX, bool FULL>
__device__ __forceinline__ double left_of(const double (&v)[PMAX], int j, double hl) {
  return j == 0 ? hl : v[j > 0 ? j - 1 : 0];
}
template <int PMAX, bool FULL>
__device__ __forceinline__ double right_of(const double (&v)[PMAX], int j, int cnt, double hr) {
  return slot_last<PMAX, FULL>(j, cnt) ? hr : v[j + 1 < PMAX ? j + 1 : PMAX - 1];
}

// Value in the chunk's last active slot.  For ragged chunks a sum of masked
// terms: a select chain over the slots is turned by the compiler into a
// dynamic register index, which moves the whole array to scratch memory.
template <int PMAX, bool FULL>
__device__ __forceinline__ double last_of(const double (&v)[PMAX], int cnt) {
  if (FULL) return v[PMAX - 1];
  double r = 0.0;
#pragma unroll
  for (int j = kMinRows<PMAX> - 1; j < PMAX; ++j) r = fma(j == cnt - 1 ? 1.0 : 0.0, v[j], r);
  return r;
}

// ds_bpermute of a double: every lane reads `v` of lane `src` (0..63).
__device__ __forceinline__ double bperm_f64(double v, int src) {
  const int lo = __builtin_amdgcn_ds_bpermute(src << 2, __double2loint(v));
  const int hi = __builtin_amdgcn_ds_bpermute(src << 2, __double2hiint(v));
  return __hiloint2double(hi, lo);
}

// Periodic neighbour exchange of K values per thread: thread t receives
// last[i] of thread t-1 in fromL[i] and first[i] of thread t+1 in fromR[i]
// (indices mod NT).  Inside a wavefront by whole-wave DPP shifts; the
// wavefront ends go through LDS (one barrier) or, for a single wavefront,
// through readlane.  The edge buffers alternate between calls (hs toggles),
// so a buffer is rewritten only after the barrier of the exchange in between.
template <int NT, int K>
__device__ __forceinline__ void exchange(const double (&first)[K], const double (&last)[K],
                                         double (&fromL)[K], double (&fromR)[K], RowLds<NT>& L,
                                         int t, int& hs) {
  constexpr int W = NT / kWave;
  static_assert(K <= 3, "at most three values per exchange");
  const int lane = t & (kWave - 1);
#pragma unroll
  for (int i = 0; i < K; ++i) {
    fromL[i] = dpp_f64z<kDppWaveShr1>(last[i]);
    fromR[i] = dpp_f64z<kDppWaveShl1>(first[i]);
  }
  if constexpr (W == 1) {
#pragma unroll
    for (int i = 0; i < K; ++i) {
      const double wl = readlane_f64(last[i], kWave - 1), wr = readlane_f64(first[i], 0);
      fromL[i] = lane == 0 ? wl : fromL[i];
      fromR[i] = lane == kWave - 1 ? wr : fromR[i];
    }
  } else {
    const int w = t / kWave;
    if (lane == kWave - 1) {
#pragma unroll
      for (int i = 0; i < K; ++i) L.edge[hs][w][2 * i + 1] = last[i];
    }
    if (lane == 0) {
#pragma unroll
      for (int i = 0; i < K; ++i) L.edge[hs][w][2 * i] = first[i];
    }
    __syncthreads();
    const int wl = (w + W - 1) & (W - 1), wr = (w + 1) & (W - 1);
#pragma unroll
    for (int i = 0; i < K; ++i) {
      const double a = L.edge[hs][wl][2 * i + 1], b = L.edge[hs][wr][2 * i];
      fromL[i] = lane == 0 ? a : fromL[i];
      fromR[i] = lane == kWave - 1 ? b : fromR[i];
    }
    hs ^= 1;
  }
}

// Left and right neighbours of the chunk (periodic).
template <int PMAX, int NT, bool FULL>
__device__ __forceinline__ void halo(const double (&v)[PMAX], int cnt, RowLds<NT>& L, int t,
                                     double& hl, double& hr, int& hs) {
  const double f[1] = {v[0]}, l[1] = {last_of<PMAX, FULL>(v, cnt)};
  double a[1], b[1];
  exchange<NT, 1>(f, l, a, b, L, t, hs);
  hl = a[0];
  hr = b[0];
}

// Partition elimination of the rows 1..E-1 of a run of E consecutive rows
// whose first unknown z_0 and whose successor z_E (the next run's z_0) are
// kept: on exit z_j = y[j] + g[j] z_0 + k[j] z_E for j = 1..E-1.  The
// coefficient arrays are indexed by the run's rows.
// `grow` receives the running maximum of the eliminated super-diagonal
// |c'_j| = |C_j / pivot_j| (see cyclic_solve).
template <int E>
__device__ __forceinline__ void spike_eliminate(const double (&A)[E], const double (&B)[E],
                                                const double (&C)[E], const double (&R)[E],
                                                double (&y)[E], double (&g)[E], double (&k)[E],
                                                double& grow) {
  double cp[E];
  double cprev = 0.0, yprev = 0.0, gprev = 1.0;
#pragma unroll
  for (int j = 1; j < E; ++j) {
    const double inv = rcp64(j == 1 ? B[j] : B[j] - A[j] * cprev);
    cp[j] = C[j] * inv;
    grow = vmax_abs(grow, cp[j]);
    y[j] = (j == 1 ? R[j] : R[j] - A[j] * yprev) * inv;
    g[j] = (j == 1 ? -A[j] : -A[j] * gprev) * inv;
    cprev = cp[j];
    yprev = y[j];
    gprev = g[j];
  }
  double yn = 0.0, gn = 0.0, kn = 1.0;
#pragma unroll
  for (int j = E - 1; j >= 1; --j) {
    y[j] = y[j] - cp[j] * yn;
    g[j] = g[j] - cp[j] * gn;
    k[j] = -cp[j] * kn;
    yn = y[j];
    gn = g[j];
    kn = k[j];
  }
}

// Solve of the periodic tridiagonal interface system of the NT chunks,
//   A_t s_{t-1} + B_t s_t + C_t s_{t+1} = R_t   (t mod NT),
// redundantly by every wavefront: lane l holds the E = NT/64 consecutive
// equations E l .. E l + E - 1 in eA..eR, eliminates all but the first by
// the partition method, and the 64 remaining equations (one per lane,
// periodic) are solved by cyclic reduction across the lanes (ds_bpermute),
// stopping once every coupling is below 2^-60 of its diagonal.  Returns, for
// the calling thread t = 64 w + lane, s_t, s_{t+1} and s_{t-1}.
template <int NT>
__device__ __forceinline__ void interface_solve(const double (&eA)[NT / kWave],
                                                const double (&eB)[NT / kWave],
                                                const double (&eC)[NT / kWave],
                                                const double (&eR)[NT / kWave], int t, double& s,
                                                double& snext, double& sprev, double& grow) {
  constexpr int E = NT / kWave;
  const int lane = t & (kWave - 1);
  double y[E], g[E], k[E];
  y[0] = 0.0;
  g[0] = 1.0;
  k[0] = 0.0;
  spike_eliminate<E>(eA, eB, eC, eR, y, g, k, grow);
  // run tails: the last unknown in terms of (z_0, z_E); first interior row
  const double yT = E > 1 ? y[E - 1] : 0.0, gT = E > 1 ? g[E - 1] : 1.0,
               kT = E > 1 ? k[E - 1] : 0.0;
  const double y1 = E > 1 ? y[1 < E ? 1 : 0] : 0.0, g1 = E > 1 ? g[1 < E ? 1 : 0] : 0.0,
               k1 = E > 1 ? k[1 < E ? 1 : 0] : 1.0;
  // tails of lane l-1 (periodic over the 64 lanes)
  double pY = dpp_f64z<kDppWaveShr1>(yT), pG = dpp_f64z<kDppWaveShr1>(gT),
         pK = dpp_f64z<kDppWaveShr1>(kT);
  {
    const double wy = readlane_f64(yT, kWave - 1), wg = readlane_f64(gT, kWave - 1),
                 wk = readlane_f64(kT, kWave - 1);
    pY = lane == 0 ? wy : pY;
    pG = lane == 0 ? wg : pG;
    pK = lane == 0 ? wk : pK;
  }
  double A = eA[0] * pG;
  double B = fma(eA[0], pK, fma(eC[0], g1, eB[0]));
  double C = eC[0] * k1;
  double R = fma(-eA[0], pY, fma(-eC[0], y1, eR[0]));
  double z = 0.0;
  {
    bool done = false;
#pragma unroll 1
    for (int d = 1; d < kWave; d <<= 1) {
      if (!__any(fabs(A) + fabs(C) > 0x1.0p-60 * fabs(B))) {
        z = R * rcp64(B);
        done = true;
        break;
      }
      const int lm = (lane - d) & (kWave - 1), lp = (lane + d) & (kWave - 1);
      const double Am = bperm_f64(A, lm), Bm = bperm_f64(B, lm), Cm = bperm_f64(C, lm),
                   Rm = bperm_f64(R, lm);
      const double Ap = bperm_f64(A, lp), Bp = bperm_f64(B, lp), Cp = bperm_f64(C, lp),
                   Rp = bperm_f64(R, lp);
      const double q1 = A * rcp64(Bm), q2 = C * rcp64(Bp);
      const double nA = -q1 * Am;
      const double nB = B - q1 * Cm - q2 * Ap;
      const double nC = -q2 * Cp;
      const double nR = R - q1 * Rm - q2 * Rp;
      A = nA;
      B = nB;
      C = nC;
      R = nR;
    }
    // after every level each equation couples z_l to itself only
    if (!done) z = R * rcp64(A + B + C);
  }
  // the run's unknowns
  const double zn = [&] {
    const double v = dpp_f64z<kDppWaveShl1>(z), w0 = readlane_f64(z, 0);
    return lane == kWave - 1 ? w0 : v;
  }();
  double zr[E];
  zr[0] = z;
#pragma unroll
  for (int e = 1; e < E; ++e) zr[e] = fma(k[e], zn, fma(g[e], z, y[e]));
  // thread t = 64 w + lane owns unknown t, held by lane t / E, slot lane % E
  const int wu = __builtin_amdgcn_readfirstlane(t / kWave);
  const int src = (kWave / E) * wu + lane / E;
  double sv = zr[0];
  if constexpr (E > 1) {
    sv = bperm_f64(zr[0], src);
#pragma unroll
    for (int e = 1; e < E; ++e) {
      const double v = bperm_f64(zr[e], src);
      sv = (lane % E) == e ? v : sv;
    }
  }
  s = sv;
  {
    const double v = dpp_f64z<kDppWaveShl1>(sv);
    const double w = readlane_f64(zr[0], ((kWave / E) * (wu + 1)) & (kWave - 1));
    snext = lane == kWave - 1 ? w : v;
  }
  {
    const double v = dpp_f64z<kDppWaveShr1>(sv);
    const double w = readlane_f64(zr[E - 1], ((kWave / E) * wu + kWave - 1) & (kWave - 1));
    sprev = lane == 0 ? w : v;
  }
}

// Workgroup solve of the periodic tridiagonal system
//     a_i x_{i-1} + b_i x_i + c_i x_{i+1} = d_i   (indices mod nx)
// distributed as chunks of rows per thread.  Partition method: the first row
// of every chunk is an interface unknown s_t; each thread eliminates its
// remaining rows by Thomas' algorithm into x_j = y_j + g_j s_t + k_j s_{t+1}
// (two spike columns), the interface rows form a periodic tridiagonal system
// of NT unknowns solved by interface_solve() behind one barrier, and the
// chunk is recombined.  row(j, a, b, c) returns the coefficients of local
// slot j and d(j) its right-hand side (both evaluated once per slot).  xl and
// xr receive the solution at the row before the chunk and the row after it
// (the halo of x, from the interface values, without another exchange).
//
// No pivoting.  The mass and Helmholtz matrices are symmetric positive
// definite and diagonally dominant.  A row of the implicit-midpoint matrix,
// (o - v_-, d + v_+ - v_-, o + v_+) with o = h/6 - mu dt/(2h),
// d = 2h/3 + mu dt/h (so d + 2o = h) and v_-+ = dv_{i-+1}/4, is diagonally
// dominant whenever |dv| / 4 <= |o| everywhere and, for o < 0, the
// compression dv_{i-1} - dv_{i+1} stays below 2h; without pivoting the LU
// factors then satisfy |L||U| <= 3|A|.  Outside that range (steep or very
// large dv) the elimination can still be accurate, and its growth is
// measured instead: row j of |L||U| is bounded by |A|'s row plus
// 2 |a_j| |c'_{j-1}|, c'_j = c_j / pivot_j the eliminated super-diagonal, so
// the solution's error grows about like max |c'| times the unit roundoff
// (near-zero pivots of a compressive saw-tooth dv: max |c'| = 250 gives a
// relative error of 1e-14, 2.5e5 gives 6e-13, 2.5e8 gives 6e-10).  `grow`
// receives the running maximum of |c'_j| over the chunk's rows and the
// interface elimination, and callers reject a system whose growth exceeds
// kMaxGrowth = 2^16 (errors below about 1e-12).
constexpr double kMaxGrowth = 65536.0;
#ifndef SCH_SWEEP_FENCE
#define SCH_SWEEP_FENCE 4
#endif
template <int PMAX, int NT, bool FULL, class RowF, class DF>
__device__ __forceinline__ void cyclic_solve(RowF row, DF d, double (&x)[PMAX], int cnt,
                                             RowLds<NT>& L, int t, double& xl, double& xr,
                                             double& grow) {
  static_assert(PMAX >= 2, "need at least two rows per thread");
  constexpr int W = NT / kWave;
  const int lane = t & (kWave - 1);
  double cp[PMAX], g[PMAX];
  // forward elimination over the interior slots 1..cnt-1; inactive slots
  // (j >= cnt) are given c' = -1, y' = g' = 0 so the back sweep passes the
  // right-spike seed (k = 1) and zeros through them unchanged.
  double cprev = 0.0, yprev = 0.0, gprev = 1.0;
#pragma unroll
  for (int j = 1; j < PMAX; ++j) {
    double a, b, c;
    row(j, a, b, c);
    // slot 1 starts the recurrences (c' = y' = 0, g' = 1 before it)
    const double inv = rcp64(j == 1 ? b : b - a * cprev);
    double cj = c * inv, yj = (j == 1 ? d(j) : d(j) - a * yprev) * inv,
           gj = (j == 1 ? -a : -a * gprev) * inv;
    if (!slot_live<PMAX, FULL>(j, cnt)) {
      cj = -1.0;
      yj = 0.0;
      gj = 0.0;
    }
    grow = vmax_abs(grow, cj);
    cp[j] = cj;
    x[j] = yj;
    g[j] = gj;
    cprev = cj;
    yprev = yj;
    gprev = gj;
    // bound the scheduler's look-ahead: rows hoisted from far ahead of the
    // recurrence would each hold four registers pairs
    if (j % SCH_SWEEP_FENCE == 0) __builtin_amdgcn_sched_barrier(0);
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
    if (!FULL && slot_last<PMAX, FULL>(j, cnt)) {
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
  // interface equation of chunk t: a0 x_{-1} + b0 s_t + c0 x_1 = d0 with
  // x_{-1} = ypl + gpl s_{t-1} + kpl s_t (thread t-1's last row) and
  // x_1 = yn + gn s_t + kn s_{t+1}
  double ypl = dpp_f64z<kDppWaveShr1>(yL), gpl = dpp_f64z<kDppWaveShr1>(gL),
         kpl = dpp_f64z<kDppWaveShr1>(kL);
  double a0, b0, c0;
  row(0, a0, b0, c0);
  const double Bp = fma(c0, gn, b0), Rp = fma(-c0, yn, d(0)), C = c0 * kn;
  double s, snext, sprev;
  if constexpr (W == 1) {
    const double wy = readlane_f64(yL, kWave - 1), wg = readlane_f64(gL, kWave - 1),
                 wk = readlane_f64(kL, kWave - 1);
    ypl = lane == 0 ? wy : ypl;
    gpl = lane == 0 ? wg : gpl;
    kpl = lane == 0 ? wk : kpl;
    const double eA[1] = {a0 * gpl}, eB[1] = {fma(a0, kpl, Bp)}, eC[1] = {C},
                 eR[1] = {fma(-a0, ypl, Rp)};
    interface_solve<NT>(eA, eB, eC, eR, t, s, snext, sprev, grow);
  } else {
    // the equation of each wavefront's first chunk goes to LDS without its
    // left-tail terms (A holds a0); the reader completes it from L.etail
    const int w = t / kWave;
    const bool firstlane = lane == 0;
    const int pt = eq_pos<NT>(t);
    L.eq[0][pt] = firstlane ? a0 : a0 * gpl;
    L.eq[1][pt] = firstlane ? Bp : fma(a0, kpl, Bp);
    L.eq[2][pt] = C;
    L.eq[3][pt] = firstlane ? Rp : fma(-a0, ypl, Rp);
    if (lane == kWave - 1) {
      L.etail[0][w] = yL;
      L.etail[1][w] = gL;
      L.etail[2][w] = kL;
    }
    __syncthreads();
    {
      const int wp = (w + W - 1) & (W - 1);
      const double ty = L.etail[0][wp], tg = L.etail[1][wp], tk = L.etail[2][wp];
      ypl = firstlane ? ty : ypl;
      gpl = firstlane ? tg : gpl;
      kpl = firstlane ? tk : kpl;
    }
    double eA[W], eB[W], eC[W], eR[W];
#pragma unroll
    for (int e = 0; e < W; ++e) {
      eA[e] = L.eq[0][e * 65 + lane];
      eB[e] = L.eq[1][e * 65 + lane];
      eC[e] = L.eq[2][e * 65 + lane];
      eR[e] = L.eq[3][e * 65 + lane];
    }
    {
      // equation W*lane is the first of a wavefront when (W*lane) % 64 == 0
      const int wq = ((W * lane) / kWave + W - 1) & (W - 1);
      const double ty = L.etail[0][wq], tg = L.etail[1][wq], tk = L.etail[2][wq];
      const bool first = ((W * lane) & (kWave - 1)) == 0;
      const double a = eA[0];
      eA[0] = first ? a * tg : eA[0];
      eB[0] = first ? fma(a, tk, eB[0]) : eB[0];
      eR[0] = first ? fma(-a, ty, eR[0]) : eR[0];
    }
    interface_solve<NT>(eA, eB, eC, eR, t, s, snext, sprev, grow);
  }
  // last row of chunk t-1: y + g s_{t-1} + k s_t with its tail values
  xl = fma(kpl, s, fma(gpl, sprev, ypl));
  xr = snext;
  x[0] = s;
  double kr = 1.0;
#pragma unroll
  for (int j = PMAX - 1; j >= 1; --j) {
    kr *= -cp[j];
    x[j] = x[j] + g[j] * s + kr * snext;
  }
}

// The same for the constant symmetric positive definite systems (no growth
// to watch).
template <int PMAX, int NT, bool FULL, class RowF, class DF>
__device__ __forceinline__ void cyclic_solve(RowF row, DF d, double (&x)[PMAX], int cnt,
                                             RowLds<NT>& L, int t, double& xl, double& xr) {
  double grow = 0.0;
  cyclic_solve<PMAX, NT, FULL>(row, d, x, cnt, L, t, xl, xr, grow);
}

// Workgroup-wide max of two values and bitwise or of small nonnegative flags.
template <int NT>
__device__ __forceinline__ void block_max2_or(double& a, double& b, int& f, RowLds<NT>& L, int t) {
  a = wave_max(a);
  b = wave_max(b);
  f = wave_or(f);
  const int w = t / kWave;
  if ((t & (kWave - 1)) == 0) {
    L.red[0][w] = a;
    L.red[1][w] = b;
    L.red[2][w] = static_cast<double>(f);
  }
  __syncthreads();
  a = L.red[0][0];
  b = L.red[1][0];
  int ff = static_cast<int>(L.red[2][0]);
#pragma unroll
  for (int i = 1; i < NT / kWave; ++i) {
    a = fmax(a, L.red[0][i]);
    b = fmax(b, L.red[1][i]);
    ff |= static_cast<int>(L.red[2][i]);
  }
  f = ff;
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
