// batch_abi.hpp -- C-ABI of the batched runner (sch_batch_*): layout of the
// batch in the caller's workspace, tile classes and their work queues, one
// cycle as a sequence of batched launches, and its capture into a HIP graph.
// Part of the abi.hip translation unit (included at its end).
#pragma once

#include <algorithm>
#include <numeric>
#include <vector>

#include "adjoint.hpp"
#include "batch.hpp"
#include "host.hpp"

struct sch_batch {
  int n_inst = 0, G = 0, n_steps = 0, n_modes = 0;
  BatchDev dev{};
  InstDev* inst_dev = nullptr;
  struct Class {
    int nt, pmax, first, count, grid;
    unsigned int* queue;
  };
  std::vector<Class> classes;
  int* items = nullptr;
  unsigned int* cycle = nullptr;
  unsigned int* queues = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

using namespace sch;


// Tile of one instance: the threads the caller asked for, else the model
// calls' choice; nodes per thread 4, 8 or 16 (the batched kernels take
// ragged chunks, so a 2-slot choice runs on 4 slots).
bool batch_tile(const sch_instance& in, Tile& tl) {
  if (in.threads == 0) {
    if (!pick_tile(in.nx, tl)) return false;
  } else {
    const int nt = in.threads;
    if (nt < 64 || nt > 512 || (nt & (nt - 1)) != 0 || in.nx < nt || (in.nx + nt - 1) / nt > 16)
      return false;
    tl = tile_for(in.nx, nt);
  }
  if (tl.pmax < 4) {
    tl.pmax = 4;
    tl.full = false;
  }
  return tile_rows_ok(in.nx, tl);
}

struct Layout {
  InstDev* inst;
  int *pinst, *items;
  unsigned int *queues, *cycle;
  double *dW, *phi, *w, *theta, *dtheta, *ess, *u0, *scratch;
  int *idx, *degenerate, *resampled, *status;
  unsigned long long *cum, *acc;
  size_t bytes;
};

Layout carve_batch(void* base, int n_inst, int64_t G, int n_steps, int n_modes, int64_t state) {
  Carve c(base);
  Layout L{};
  L.inst = c.take<InstDev>(n_inst);
  L.pinst = c.take<int>(G);
  L.items = c.take<int>(G);
  L.queues = c.take<unsigned int>(16);
  L.cycle = c.take<unsigned int>(1);
  L.dW = c.take<double>(G * n_steps * n_modes);
  L.phi = c.take<double>(G);
  L.w = c.take<double>(G);
  L.theta = c.take<double>(n_inst);
  L.dtheta = c.take<double>(n_inst);
  L.ess = c.take<double>(n_inst);
  L.u0 = c.take<double>(n_inst);
  L.idx = c.take<int>(G);
  L.degenerate = c.take<int>(n_inst);
  L.resampled = c.take<int>(n_inst);
  L.status = c.take<int>(G);
  L.cum = c.take<unsigned long long>(G);
  L.scratch = c.take<double>(state);
  L.acc = c.take<unsigned long long>(1);
  L.bytes = c.off + 256;
  return L;
}

int check_batch(const sch_batch_params* bp, int n_inst, const sch_instance* in, int64_t& G,
                int64_t& state) {
  if (!bp || n_inst < 1 || !in) return fail(SCH_E_ARG, "bad arguments to the batched runner");
  if (!(bp->L > 0) || !(bp->alpha > 0) || !(bp->mu >= 0) || !(bp->dt > 0) || bp->n_modes < 1 ||
      bp->n_modes > 64 || bp->n_steps < 1 || bp->n_obs < 1 || !(bp->picard_tol > 0) ||
      bp->picard_max < 1 || !(bp->ess_frac >= 0))
    return fail(SCH_E_ARG, "bad batch parameters");
  G = 0;
  state = 0;
  for (int i = 0; i < n_inst; ++i) {
    const sch_instance& s = in[i];
    Tile tl;
    if (s.nx < 64 || s.nx > 8192 || s.n_particles < 1 || s.n_particles > 65536)
      return fail(SCH_E_SHAPE, "instance %d: nx = %d, n = %d not supported", i, s.nx,
                  s.n_particles);
    if (!batch_tile(s, tl))
      return fail(SCH_E_SHAPE, "instance %d: no tile for nx = %d with %d threads", i, s.nx,
                  s.threads);
    G += s.n_particles;
    state += static_cast<int64_t>(s.n_particles) * 2 * s.nx;
  }
  if (G > (1 << 30)) return fail(SCH_E_SHAPE, "too many particles in the batch");
  return SCH_OK;
}

template <class F>
int with_batch_class(int nt, int pm, F&& f) {
#define SCH_BCASE(NT_, PM_) \
  if (nt == NT_ && pm == PM_) return f.template operator()<PM_, NT_>();
  SCH_BCASE(64, 4) SCH_BCASE(64, 8) SCH_BCASE(64, 16)
  SCH_BCASE(128, 4) SCH_BCASE(128, 8) SCH_BCASE(128, 16)
  SCH_BCASE(256, 4) SCH_BCASE(256, 8) SCH_BCASE(256, 16)
  SCH_BCASE(512, 4) SCH_BCASE(512, 8) SCH_BCASE(512, 16)
#undef SCH_BCASE
  return fail(SCH_E_SHAPE, "no batched kernel for %d threads x %d nodes", nt, pm);
}

// One assimilation cycle of every instance, enqueued on `st`.  `timed`
// brackets the kernel classes with timing events (direct launches only, not
// under graph capture).
int enqueue_cycle(sch_batch* b, hipStream_t st, bool timed) {
  const BatchDev& B = b->dev;
  auto scope = [&](int kind) { return TimedScope(timed ? kind : -1, st); };
  {
    auto ts = scope(SCH_TK_OTHER);
    for (auto& c : b->classes)
      hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, c.queue, 0u, 1);
    const int64_t work = static_cast<int64_t>(b->G) * b->n_steps * ((b->n_modes + 1) / 2);
    hipLaunchKernelGGL(k_batch_draw, dim3(grid_for(work, 256)), dim3(256), 0, st, B);
  }
  {
    auto ts = scope(SCH_TK_WINDOW);
    for (auto& c : b->classes) {
      const int* items = b->items + c.first;
      const int n_items = c.count;
      unsigned int* q = c.queue;
      const int grid = c.grid;
      if (int rc = with_batch_class(c.nt, c.pmax, [&]<int PM, int NT>() -> int {
            hipLaunchKernelGGL((k_batch_window<PM, NT>), dim3(grid), dim3(NT), 0, st, B, items,
                               n_items, q);
            return SCH_OK;
          }))
        return rc;
    }
  }
  {
    auto ts = scope(SCH_TK_OTHER);
    hipLaunchKernelGGL(k_batch_loglik, dim3(b->G), dim3(kWave), 0, st, B);
  }
  {
    auto ts = scope(SCH_TK_TEMPER);
    hipLaunchKernelGGL(k_batch_weights, dim3(b->n_inst), dim3(kTB), 0, st, B);
  }
  {
    auto ts = scope(SCH_TK_RESAMPLE);
    hipLaunchKernelGGL(k_batch_resample, dim3(b->n_inst), dim3(kTB), 0, st, B);
  }
  {
    auto ts = scope(SCH_TK_GATHER);
    hipLaunchKernelGGL(k_batch_gather, dim3(b->G), dim3(256), 0, st, B, 0);
    hipLaunchKernelGGL(k_batch_gather, dim3(b->G), dim3(256), 0, st, B, 1);
  }
  hipLaunchKernelGGL(k_batch_next_cycle, dim3(1), dim3(64), 0, st, b->cycle);
  CHECK_LAUNCH();
  return SCH_OK;
}

}  // namespace


extern "C" {

size_t sch_batch_workspace_bytes(const sch_batch_params* bp, int32_t n_inst,
                                 const sch_instance* in) {
  int64_t G = 0, state = 0;
  if (check_batch(bp, n_inst, in, G, state) != SCH_OK) return 0;
  return carve_batch(nullptr, n_inst, G, bp->n_steps, bp->n_modes, state).bytes;
}

int sch_batch_create(const sch_batch_params* bp, int32_t n_inst, const sch_instance* in,
                     void* workspace, size_t bytes, sch_batch** out, void* stream) {
  int64_t G = 0, state = 0;
  if (int rc = check_batch(bp, n_inst, in, G, state)) return rc;
  if (!workspace || !out) return fail(SCH_E_ARG, "bad arguments to sch_batch_create");
  for (int i = 0; i < n_inst; ++i)
    if (!in[i].xi || !in[i].m || !in[i].u || !in[i].logw || !in[i].y || !in[i].sigma)
      return fail(SCH_E_ARG, "instance %d has a NULL array", i);
  Layout L = carve_batch(workspace, n_inst, G, bp->n_steps, bp->n_modes, state);
  if (bytes < L.bytes) return fail(SCH_E_ARG, "workspace of %zu bytes < %zu", bytes, L.bytes);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);

  // per-instance table and the particle -> instance map
  std::vector<InstDev> inst(n_inst);
  std::vector<int> pinst(G);
  std::vector<Tile> tiles(n_inst);
  int64_t g0 = 0, s0 = 0;
  for (int i = 0; i < n_inst; ++i) {
    const sch_instance& s = in[i];
    batch_tile(s, tiles[i]);
    sch_model md{bp->L, bp->alpha, bp->mu, bp->dt, s.nx, bp->n_modes, s.xi, bp->picard_tol,
                 bp->picard_max};
    InstDev& D = inst[i];
    D.P = make_params(md);
    D.K = make_helm(md, tiles[i]);
    D.m = s.m;
    D.u = s.u;
    D.logw = s.logw;
    D.y = s.y;
    D.sigma = s.sigma;
    D.seed = s.seed;
    D.n = s.n_particles;
    D.n_obs = bp->n_obs;
    D.g0 = g0;
    D.s0 = s0;
    D.thr = bp->ess_frac * s.n_particles;
    for (int p = 0; p < s.n_particles; ++p) pinst[g0 + p] = i;
    g0 += s.n_particles;
    s0 += static_cast<int64_t>(s.n_particles) * 2 * s.nx;
  }
  // tile classes; within a class the largest grids first (longest jobs first)
  auto b = new sch_batch();
  b->n_inst = n_inst;
  b->G = static_cast<int>(G);
  b->n_steps = bp->n_steps;
  b->n_modes = bp->n_modes;
  std::vector<int> order(n_inst);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
    if (tiles[a].nt != tiles[c].nt) return tiles[a].nt > tiles[c].nt;
    if (tiles[a].pmax != tiles[c].pmax) return tiles[a].pmax > tiles[c].pmax;
    return in[a].nx > in[c].nx;
  });
  std::vector<int> items;
  items.reserve(G);
  int dev = 0, n_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
    delete b;
    return fail(SCH_E_HIP, "cannot query the device");
  }
  for (int k = 0; k < n_inst;) {
    const int nt = tiles[order[k]].nt, pm = tiles[order[k]].pmax;
    sch_batch::Class c{nt, pm, static_cast<int>(items.size()), 0, 0, nullptr};
    while (k < n_inst && tiles[order[k]].nt == nt && tiles[order[k]].pmax == pm) {
      const int i = order[k];
      for (int p = 0; p < in[i].n_particles; ++p) items.push_back(static_cast<int>(inst[i].g0 + p));
      ++k;
    }
    c.count = static_cast<int>(items.size()) - c.first;
    if (b->classes.size() >= 16) {
      delete b;
      return fail(SCH_E_SHAPE, "too many tile classes");
    }
    c.queue = L.queues + b->classes.size();
    int per_cu = 1;
    int rc = with_batch_class(nt, pm, [&]<int PM, int NT>() -> int {
      int nb = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch_window<PM, NT>, NT, 0) !=
          hipSuccess)
        return fail(SCH_E_HIP, "occupancy query failed");
      per_cu = std::max(nb, 1);
      return SCH_OK;
    });
    if (rc) {
      delete b;
      return rc;
    }
    c.grid = static_cast<int>(std::min<int64_t>(c.count, static_cast<int64_t>(n_cu) * per_cu));
    b->classes.push_back(c);
  }
  b->inst_dev = L.inst;
  b->items = L.items;
  b->cycle = L.cycle;
  b->queues = L.queues;
  BatchDev& B = b->dev;
  B.inst = L.inst;
  B.pinst = L.pinst;
  B.G = b->G;
  B.n_inst = n_inst;
  B.n_steps = bp->n_steps;
  B.n_modes = bp->n_modes;
  B.cycle = L.cycle;
  B.dW = L.dW;
  B.phi = L.phi;
  B.w = L.w;
  B.theta = L.theta;
  B.dtheta = L.dtheta;
  B.ess = L.ess;
  B.u0 = L.u0;
  B.idx = L.idx;
  B.degenerate = L.degenerate;
  B.resampled = L.resampled;
  B.status = L.status;
  B.cum = L.cum;
  B.scratch = L.scratch;
  B.acc = L.acc;
  auto cleanup = [&](int rc) {
    delete b;
    return rc;
  };
  if (hipMemcpyAsync(L.inst, inst.data(), sizeof(InstDev) * n_inst, hipMemcpyHostToDevice, st) !=
          hipSuccess ||
      hipMemcpyAsync(L.pinst, pinst.data(), sizeof(int) * G, hipMemcpyHostToDevice, st) !=
          hipSuccess ||
      hipMemcpyAsync(L.items, items.data(), sizeof(int) * G, hipMemcpyHostToDevice, st) !=
          hipSuccess)
    return cleanup(fail(SCH_E_HIP, "table upload failed"));
  const int gb = grid_for(G, 256);
  hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n_inst, 256)), dim3(256), 0, st, L.resampled, 0,
                     n_inst);
  hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n_inst, 256)), dim3(256), 0, st, L.degenerate, 0,
                     n_inst);
  hipLaunchKernelGGL(k_fill_i32, dim3(gb), dim3(256), 0, st, L.status, 0, b->G);
  hipLaunchKernelGGL(k_fill, dim3(grid_for(n_inst, 256)), dim3(256), 0, st, L.ess, 0.0,
                     int64_t(n_inst));
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, L.acc, 1);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess)
    return cleanup(fail(SCH_E_HIP, "batch set-up failed"));
  *out = b;
  return SCH_OK;
}

int sch_batch_run(sch_batch* b, uint32_t cycle0, int32_t n_cycles, int32_t use_graph,
                  void* stream) {
  if (!b || n_cycles < 0) return fail(SCH_E_ARG, "bad arguments to sch_batch_run");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, b->cycle, cycle0, 1);
  CHECK_LAUNCH();
  if (!use_graph) {
    for (int c = 0; c < n_cycles; ++c)
      if (int rc = enqueue_cycle(b, st, true)) return rc;
    return SCH_OK;
  }
  if (!b->exec) {
    // capture one cycle on a stream of our own (the caller's may be the null
    // stream, which cannot be captured)
    hipStream_t cs = nullptr;
    HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      (void)hipStreamDestroy(cs);
      return fail(SCH_E_HIP, "graph capture could not start");
    }
    const int rc = enqueue_cycle(b, cs, false);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(cs, &g);
    (void)hipStreamDestroy(cs);
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess || !g) return fail(SCH_E_HIP, "graph capture failed");
    hipGraphExec_t ex = nullptr;
    if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
      (void)hipGraphDestroy(g);
      return fail(SCH_E_HIP, "graph instantiation failed");
    }
    b->graph = g;
    b->exec = ex;
  }
  for (int c = 0; c < n_cycles; ++c) HIP_TRY(hipGraphLaunch(b->exec, st));
  return SCH_OK;
}

int sch_batch_read(sch_batch* b, double* ess, int32_t* resampled, int32_t* status,
                   int64_t* picard_iters, void* stream) {
  if (!b) return fail(SCH_E_ARG, "bad arguments to sch_batch_read");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const BatchDev& B = b->dev;
  std::vector<int> gst(b->G);
  std::vector<InstDev> inst(b->n_inst);
  unsigned long long acc = 0;
  if (ess) HIP_TRY(hipMemcpyAsync(ess, B.ess, sizeof(double) * b->n_inst, hipMemcpyDeviceToHost, st));
  if (resampled)
    HIP_TRY(hipMemcpyAsync(resampled, B.resampled, sizeof(int) * b->n_inst, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(gst.data(), B.status, sizeof(int) * b->G, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(inst.data(), b->inst_dev, sizeof(InstDev) * b->n_inst,
                         hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(&acc, B.acc, sizeof acc, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  timing_flush();
  if (status)
    for (int i = 0; i < b->n_inst; ++i) {
      status[i] = SCH_OK;
      for (int p = 0; p < inst[i].n && status[i] == SCH_OK; ++p) status[i] = gst[inst[i].g0 + p];
    }
  if (picard_iters) *picard_iters = static_cast<int64_t>(acc);
  return SCH_OK;
}

int sch_batch_destroy(sch_batch* b) {
  if (!b) return SCH_OK;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  delete b;
  return SCH_OK;
}

}  // extern "C"
