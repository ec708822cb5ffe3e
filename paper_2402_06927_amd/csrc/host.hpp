// host.hpp -- host-side helpers shared by the C-ABI translation units:
// error reporting, launch checks, tile choice, Helmholtz scan constants,
// model validation and the workspace carver.
#pragma once

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <string>

#include "helm.hpp"

namespace sch {

inline thread_local std::string g_err;

inline int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(expr)                                                                 \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess) return fail(SCH_E_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

#define CHECK_LAUNCH() HIP_TRY(hipGetLastError())

inline hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

inline int grid_for(int64_t work, int block) {
  int64_t g = (work + block - 1) / block;
  if (g < 1) g = 1;
  if (g > 65536) g = 65536;
  return static_cast<int>(g);
}

// ---------------------------------------------------------------------------
// Tile choice: NT threads per particle (power of two, 64..512), each holding
// up to PMAX consecutive nodes in registers (tile_for).  By default NT is the smallest
// power of two with nx / NT <= 8; SCH_TUNE_THREADS overrides it.
struct Tile {
  int nt, pmax;
  bool full;
};

// Slots per thread: 4, 8 or 16, and 2 on a single wavefront (nx <= 128),
// where the chunk sweeps would otherwise carry masked slots beside one or two
// rows.
inline Tile tile_for(int nx, int nt) {
  Tile tl{};
  tl.nt = nt;
  const int need = (nx + nt - 1) / nt;
  tl.pmax = (nt == 64 && need <= 2) ? 2 : need <= 4 ? 4 : (need <= 8 ? 8 : 16);
  tl.full = (nx % nt == 0) && (nx / nt == tl.pmax);
  return tl;
}

// The kernels take every chunk to hold at least kMinRows<PMAX> rows (their
// ragged-chunk masks start there): PMAX / 2 for 8 and 16 slots, else 1.
inline bool tile_rows_ok(int nx, const Tile& tl) {
  const int min_rows = tl.pmax >= 8 ? tl.pmax / 2 : 1;
  return nx / tl.nt >= min_rows && (nx + tl.nt - 1) / tl.nt <= tl.pmax;
}

inline int g_tune_threads = 0;  // SCH_TUNE_THREADS

inline bool pick_tile(int nx, Tile& tl) {
  if (nx < 64 || nx > 8192) return false;
  int nt = g_tune_threads;
  if (nt == 0) {
    const int per = (nx + 7) / 8;
    nt = 64;
    while (nt < per && nt < 512) nt <<= 1;
  }
  if (nx < nt || (nx + nt - 1) / nt > 16) return false;
  tl = tile_for(nx, nt);
  return tile_rows_ok(nx, tl);
}

// Constants of the scan form (helm.hpp) of the solve with M + a2 K on nx
// periodic cells of width h.
inline HelmConst make_helm_op(double h, int nx, double a2, const Tile& tl) {
  HelmConst K{};
  K.ho = h / 6.0 - a2 / h;
  K.hd = 2.0 * h / 3.0 + 2.0 * a2 / h;
  // |x| > 2 (diagonal dominance); r is the root of r^2 - x r + 1 = 0 inside
  // the unit interval, of the sign of x
  const double x = -K.hd / K.ho;
  K.r = 2.0 / (x + std::copysign(std::sqrt((x - 2.0) * (x + 2.0)), x));
  const double kappa = -K.ho / K.r;
  K.coef = 1.0 / (kappa * (1.0 - K.r) * (1.0 + K.r));
  K.rN1 = 1.0 / (1.0 - std::pow(K.r, static_cast<double>(nx)));
  K.base = nx / tl.nt;
  K.rb = std::pow(K.r, static_cast<double>(K.base));
  K.rb1 = std::pow(K.r, static_cast<double>(K.base + 1));
  K.rinv = 1.0 / K.r;
  K.mh6 = h / 6.0;
  K.mh23 = 2.0 * h / 3.0;
  const double beta = K.mh6 / K.ho, gamma = K.mh23 - beta * K.hd;
  K.mg = gamma * K.coef;
  K.mf = beta - K.mg;
  // powers of rb in the order the scan form's lane factors are built
  const double rb2 = K.rb * K.rb, rb4 = rb2 * rb2, rb8 = rb4 * rb4, rb16 = rb8 * rb8,
               rb32 = rb16 * rb16, rb64 = rb32 * rb32;
  for (int e = 0; e <= 64; ++e) {
    double p = (e & 1) ? K.rb : 1.0;
    p *= (e & 2) ? rb2 : 1.0;
    p *= (e & 4) ? rb4 : 1.0;
    p *= (e & 8) ? rb8 : 1.0;
    p *= (e & 16) ? rb16 : 1.0;
    p *= (e & 32) ? rb32 : 1.0;
    K.pwt[e] = (e & 64) ? p * rb64 : p;
  }
  return K;
}

// The Helmholtz operator H = M + alpha^2 K of the model.
inline HelmConst make_helm(const sch_model& md, const Tile& tl) {
  return make_helm_op(md.L / md.nx, md.nx, md.alpha * md.alpha, tl);
}

template <class F>
inline int with_tile(const Tile& tl, F&& f) {
#define SCH_CASE(NT_, PM_)                                                       \
  if (tl.nt == NT_ && tl.pmax == PM_)                                            \
    return tl.full ? f.template operator()<PM_, NT_, true>()                     \
                   : f.template operator()<PM_, NT_, false>();
  SCH_CASE(64, 2)
  SCH_CASE(64, 4)
  SCH_CASE(64, 8)
  SCH_CASE(64, 16)
  SCH_CASE(128, 8)
  SCH_CASE(128, 16)
  SCH_CASE(256, 8)
  SCH_CASE(256, 16)
  SCH_CASE(512, 8)
  SCH_CASE(512, 16)
#undef SCH_CASE
  return fail(SCH_E_SHAPE, "no kernel for %d threads x %d nodes", tl.nt, tl.pmax);
}


inline int check_model(const sch_model* md, Tile& tl) {
  if (!md) return fail(SCH_E_ARG, "model is NULL");
  if (!(md->L > 0) || !(md->alpha > 0) || !(md->mu >= 0) || !(md->dt > 0))
    return fail(SCH_E_ARG, "need L > 0, alpha > 0, mu >= 0, dt > 0");
  if (md->nx < 64) return fail(SCH_E_SHAPE, "nx = %d < 64", md->nx);
  if (md->n_modes < 1 || md->n_modes > 64) return fail(SCH_E_ARG, "n_modes = %d", md->n_modes);
  if (!md->xi) return fail(SCH_E_ARG, "xi is NULL");
  if (!(md->picard_tol > 0) || md->picard_max < 1)
    return fail(SCH_E_ARG, "need picard_tol > 0 and picard_max >= 1");
  if (!pick_tile(md->nx, tl)) return fail(SCH_E_SHAPE, "nx = %d not supported", md->nx);
  return SCH_OK;
}


// Bump allocator over the caller's workspace (256-byte aligned pieces).
struct Carve {
  char* base;
  size_t off = 0;
  explicit Carve(void* b) : base(static_cast<char*>(b)) {}
  template <class T>
  T* take(size_t n) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += n * sizeof(T);
    return p;
  }
};

}  // namespace sch
