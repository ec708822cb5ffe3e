// mlp_abi.hpp -- C-ABI of the warm-start network (sch_mlp_*).  Part of the
// abi.hip translation unit (included at its end).
#pragma once

#include "host.hpp"
#include "mlp.hpp"

namespace {

using namespace sch;

bool mlp_ok(const sch_mlp* n) {
  return n && n->n_in >= 1 && n->n_hidden >= 1 && n->n_out >= 1 && n->params && n->weights_bf16;
}

// Activations of the last forward pass, kept in the caller's workspace for
// the backward pass: Z1, Z2 (float32), H1, H2 (bf16), then the backward
// temporaries dY (float32, bf16), dZ2, dZ1 (float32, bf16); the transposed
// bf16 copies (...T) that put every backward product's operands contiguous
// along its summation index; the column-sum partials.
struct MlpWs {
  float *Z1, *Z2, *dY32, *dZ2, *dZ1;
  float* kpart;  // split-K partials (the first layer, the weight gradients)
  uint16_t *H1, *H2, *dY16, *dZ2b, *dZ1b;
  uint16_t *XT, *dYT, *H1T, *H2T, *dZ2T, *dZ1T, *W2T, *W3T;
  double* part;
  size_t bytes;
};

int colsum_parts(int rows) { return (rows + kColsumRows - 1) / kColsumRows; }

// Slices of K for a product on a K-contiguous loader with tm x tm tiles and
// chunks of kc values of k: when its tiles alone fill fewer than half the
// chip's 256 compute units (the first layer: 64 tiles, of 128 x 128 at 4096
// rows and of 64 x 64 at 1024; the weight gradients of the second and third
// layers: 16 and 20 tiles of 64 x 64), K is split until the slices fill it
// (at most 16, each at least 2 chunks; K a multiple of kc).
int ksplit(int M, int N, int K, int tm, int kc) {
  const int tiles = ((M + tm - 1) / tm) * ((N + tm - 1) / tm);
  if (K % kc != 0 || tiles >= 128) return 1;
  int z = 1;
  while (z < 16 && tiles * 2 * z <= 256 && K / kc >= 2 * (2 * z)) z *= 2;
  return z;
}

// The loader launch_gemm takes for a product whose operands are contiguous
// along K: long K (the first layer's products) loads straight to LDS, on
// 128 x 128 tiles where at least 64 of them cover the product (a quarter of
// the chip, so a split of at most 4 fills it: the first layer at 4096 rows,
// 31 us against 40 on 64 x 64 tiles) and on 64 x 64 tiles otherwise (at 1024
// rows 16 tiles of 128 split 16 ways took 12.3 + 7.4 us for the sum of the
// slices, 64 tiles of 64 split 4 ways 13.0 + 4.1); shorter K takes the
// register prefetch, which measured faster there.
struct GemmPlan {
  bool lds;
  int tm, kc, kz;
};
GemmPlan plan_gemm(int M, int N, int K, bool split) {
  GemmPlan p{};
  p.lds = K >= 2048 && K % kLC == 0;
  p.tm = p.lds && ((M + 127) / 128) * ((N + 127) / 128) >= 64 ? 128 : 64;
  p.kc = p.tm == 128 ? kLC / 2 : kLC;
  p.kz = split ? ksplit(M, N, K, p.tm, p.kc) : 1;
  return p;
}

MlpWs carve_mlp(void* base, const MlpDims& d, int batch) {
  Carve c(base);
  MlpWs w{};
  const size_t bh = static_cast<size_t>(batch) * d.H, bo = static_cast<size_t>(batch) * d.O;
  w.Z1 = c.take<float>(bh);
  w.Z2 = c.take<float>(bh);
  // split-K partials of the first layer and of the three weight gradients
  // (one product at a time)
  size_t kp = 0;
  const int split[4][3] = {{batch, d.H, d.F}, {d.O, d.H, batch}, {d.H, d.H, batch},
                           {d.H, d.F, batch}};
  for (const auto& p : split) {
    const int kz = plan_gemm(p[0], p[1], p[2], true).kz;
    if (kz > 1) kp = std::max(kp, static_cast<size_t>(kz) * p[0] * p[1]);
  }
  w.kpart = c.take<float>(kp);
  w.H1 = c.take<uint16_t>(bh);
  w.H2 = c.take<uint16_t>(bh);
  w.dY32 = c.take<float>(bo);
  w.dY16 = c.take<uint16_t>(bo);
  w.dZ2 = c.take<float>(bh);
  w.dZ2b = c.take<uint16_t>(bh);
  w.dZ1 = c.take<float>(bh);
  w.dZ1b = c.take<uint16_t>(bh);
  w.XT = c.take<uint16_t>(static_cast<size_t>(batch) * d.F);
  w.dYT = c.take<uint16_t>(bo);
  w.H1T = c.take<uint16_t>(bh);
  w.H2T = c.take<uint16_t>(bh);
  w.dZ2T = c.take<uint16_t>(bh);
  w.dZ1T = c.take<uint16_t>(bh);
  w.W2T = c.take<uint16_t>(static_cast<size_t>(d.H) * d.H);
  w.W3T = c.take<uint16_t>(static_cast<size_t>(d.H) * d.O);
  w.part = c.take<double>(static_cast<size_t>(colsum_parts(batch)) * (2 * d.H + d.O));
  w.bytes = c.off + 256;
  return w;
}

// Collects up to kTransposeBatch dense transposes and issues them as one launch.
struct TransposeList {
  TransposeBatch b{};
  void add(int rows, int cols, const uint16_t* in, uint16_t* out) {
    if (rows <= 0 || cols <= 0) return;
    const int k = b.n++;
    b.rows[k] = rows;
    b.cols[k] = cols;
    b.tx[k] = (cols + 63) / 64;
    b.in[k] = in;
    b.out[k] = out;
    b.tile0[k + 1] = b.tile0[k] + b.tx[k] * ((rows + 63) / 64);
  }
  void launch(hipStream_t st) const {
    if (b.n > 0)
      hipLaunchKernelGGL(k_transpose_bf16, dim3(b.tile0[b.n]), dim3(256), 0, st, b);
  }
};

// Collects up to kColsumBatch column sums over the same rows and issues them
// as one pair of launches (part: colsum_parts(rows) x the total columns).
struct ColsumList {
  ColsumBatch b{};
  void add(int cols, const float* A, float* out) {
    const int k = b.n++;
    b.cols[k] = cols;
    b.A[k] = A;
    b.out[k] = out;
    b.tile0[k + 1] = b.tile0[k] + (cols + 63) / 64;
    b.coff[k + 1] = b.coff[k] + cols;
  }
  void launch(int rows, double* part, hipStream_t st) const {
    const int nb = colsum_parts(rows);
    hipLaunchKernelGGL(k_colsum_part, dim3(b.tile0[b.n], nb), dim3(256), 0, st, rows, b, part);
    hipLaunchKernelGGL(k_colsum_final, dim3((b.coff[b.n] + 255) / 256), dim3(256), 0, st, nb, b,
                       part);
  }
};

GemmArgs gemm(int M, int N, int K, const uint16_t* A, int64_t sam, int64_t sak,
              const uint16_t* B, int64_t sbk, int64_t sbn) {
  GemmArgs g{};
  g.M = M;
  g.N = N;
  g.K = K;
  g.A = A;
  g.sam = sam;
  g.sak = sak;
  g.B = B;
  g.sbk = sbk;
  g.sbn = sbn;
  return g;
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

void launch_gemm(const GemmArgs& g, hipStream_t st) {
  // (the K-contiguous loaders clamp their reads to K - 8: K >= 8)
  const bool kc = g.sak == 1 && g.sbk == 1 && g.K >= 8 && g.K % 8 == 0 && g.sam % 8 == 0 &&
                  g.sbn % 8 == 0 && aligned16(g.A) && aligned16(g.B);
  if (!kc) {
    hipLaunchKernelGGL(k_gemm_bf16, dim3((g.N + kGN - 1) / kGN, (g.M + kGM - 1) / kGM),
                       dim3(256), 0, st, g);
    return;
  }
  // K split over idle compute units where the caller gave the partials'
  // buffer
  const GemmPlan p = plan_gemm(g.M, g.N, g.K, g.kpart != nullptr);
  const dim3 grid((g.N + p.tm - 1) / p.tm, (g.M + p.tm - 1) / p.tm, p.kz);
  if (p.lds && p.tm == 128)
    hipLaunchKernelGGL((k_gemm_bf16_lds<128>), grid, dim3(256), 0, st, g);
  else if (p.lds)
    hipLaunchKernelGGL((k_gemm_bf16_lds<64>), grid, dim3(256), 0, st, g);
  else
    hipLaunchKernelGGL((k_gemm_bf16_kc<kLC, 2>), grid, dim3(256), 0, st, g);
  if (p.kz > 1)
    hipLaunchKernelGGL(k_gemm_reduce, dim3(grid_for(static_cast<int64_t>(g.M) * g.N, 256)),
                       dim3(256), 0, st, g, p.kz);
}

}  // namespace

extern "C" {

size_t sch_mlp_param_count(int32_t n_in, int32_t n_hidden, int32_t n_out) {
  if (n_in < 1 || n_hidden < 1 || n_out < 1) return 0;
  return static_cast<size_t>(mlp_dims(n_in, n_hidden, n_out).n_params);
}

size_t sch_mlp_workspace_bytes(const sch_mlp* net, int32_t batch) {
  if (!net || net->n_in < 1 || net->n_hidden < 1 || net->n_out < 1 || batch < 1) return 0;
  return carve_mlp(nullptr, mlp_dims(net->n_in, net->n_hidden, net->n_out), batch).bytes;
}

int sch_mlp_sync(const sch_mlp* net, void* stream) {
  if (!mlp_ok(net)) return fail(SCH_E_ARG, "bad network");
  const MlpDims d = mlp_dims(net->n_in, net->n_hidden, net->n_out);
  hipLaunchKernelGGL(k_adam, dim3(grid_for(d.n_params, 256)), dim3(256), 0, S(stream), d,
                     net->params, nullptr, nullptr, nullptr, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f,
                     net->weights_bf16);
  CHECK_LAUNCH();
  return SCH_OK;
}

int sch_mlp_forward(const sch_mlp* net, int32_t batch, const uint16_t* X, float* Y,
                    void* workspace, void* stream) {
  if (!mlp_ok(net) || batch < 1 || !X || !Y || !workspace)
    return fail(SCH_E_ARG, "bad arguments to sch_mlp_forward");
  const MlpDims d = mlp_dims(net->n_in, net->n_hidden, net->n_out);
  const MlpWs w = carve_mlp(workspace, d, batch);
  hipStream_t st = S(stream);
  const float* p = net->params;
  const uint16_t* wb = net->weights_bf16;
  const int F = d.F, H = d.H, O = d.O;
  GemmArgs g = gemm(batch, H, F, X, F, 1, wb, 1, F);  // Z1 = X W1^T + b1
  g.kpart = w.kpart;
  g.bias = p + d.ob1;
  g.C32 = w.Z1;
  g.ldc = H;
  g.C16 = w.H1;
  g.ldc16 = H;
  g.relu = 1;
  launch_gemm(g, st);
  g = gemm(batch, H, H, w.H1, H, 1, wb + d.qW2, 1, H);  // Z2 = H1 W2^T + b2
  g.bias = p + d.ob2;
  g.C32 = w.Z2;
  g.ldc = H;
  g.C16 = w.H2;
  g.ldc16 = H;
  g.relu = 1;
  launch_gemm(g, st);
  g = gemm(batch, O, H, w.H2, H, 1, wb + d.qW3, 1, H);  // Y = H2 W3^T + b3
  g.bias = p + d.ob3;
  g.C32 = Y;
  g.ldc = O;
  launch_gemm(g, st);
  CHECK_LAUNCH();
  return SCH_OK;
}

int sch_mlp_backward(const sch_mlp* net, int32_t batch, const uint16_t* X, const float* Y,
                     const float* T, double* loss, float* grad, void* workspace, void* stream) {
  if (!mlp_ok(net) || batch < 1 || !X || !Y || !T || !loss || !grad || !workspace)
    return fail(SCH_E_ARG, "bad arguments to sch_mlp_backward");
  const MlpDims d = mlp_dims(net->n_in, net->n_hidden, net->n_out);
  const MlpWs w = carve_mlp(workspace, d, batch);
  hipStream_t st = S(stream);
  const uint16_t* wb = net->weights_bf16;
  const int F = d.F, H = d.H, O = d.O;
  const int64_t bo = static_cast<int64_t>(batch) * O;
  hipLaunchKernelGGL(k_fill, dim3(1), dim3(64), 0, st, loss, 0.0, int64_t(1));
  // at most 128 workgroups: each adds its share to *loss with one atomic, and
  // atomics on one address serialise
  hipLaunchKernelGGL(k_mse, dim3(std::min(grid_for(bo, 256), 128)), dim3(256), 0, st, bo, Y, T,
                     1.0f / static_cast<float>(bo), w.dY32, w.dY16, loss);
  // Every product below runs with both operands contiguous along its sum
  // (the fast loader): the weights W2, W3 are transposed once per call, and
  // for a batch that is a multiple of 8 the activations and X are too, so the
  // weight gradients (summed over the batch) take that loader as well;
  // otherwise those take the element-wise loader on the original layouts.
  // Transposing moves bf16 values unchanged: the products' rounding is the
  // same either way.
  const bool tr = batch % 8 == 0;
  TransposeList tl;
  tl.add(H, H, wb + d.qW2, w.W2T);
  tl.add(O, H, wb + d.qW3, w.W3T);
  if (tr) {
    tl.add(batch, O, w.dY16, w.dYT);
    tl.add(batch, H, w.H2, w.H2T);
    tl.add(batch, H, w.H1, w.H1T);
    tl.add(batch, F, X, w.XT);
  }
  tl.launch(st);
  // the bias gradients (column sums of dY, dZ2, dZ1) run together at the end
  ColsumList cs;
  // dW3 = dY^T H2, db3 = column sums of dY
  GemmArgs g = tr ? gemm(O, H, batch, w.dYT, batch, 1, w.H2T, 1, batch)
                  : gemm(O, H, batch, w.dY16, 1, O, w.H2, H, 1);
  g.C32 = grad + d.oW3;
  g.ldc = H;
  g.kpart = w.kpart;
  launch_gemm(g, st);
  cs.add(O, w.dY32, grad + d.ob3);
  // dZ2 = (dY W3) * [Z2 > 0]
  g = gemm(batch, H, O, w.dY16, O, 1, w.W3T, 1, O);
  g.mask = w.Z2;
  g.ldm = H;
  g.C32 = w.dZ2;
  g.ldc = H;
  g.C16 = w.dZ2b;
  g.ldc16 = H;
  if (tr) {
    g.C16T = w.dZ2T;
    g.ldt = batch;
  }
  launch_gemm(g, st);
  // dW2 = dZ2^T H1, db2
  g = tr ? gemm(H, H, batch, w.dZ2T, batch, 1, w.H1T, 1, batch)
         : gemm(H, H, batch, w.dZ2b, 1, H, w.H1, H, 1);
  g.C32 = grad + d.oW2;
  g.ldc = H;
  g.kpart = w.kpart;
  launch_gemm(g, st);
  cs.add(H, w.dZ2, grad + d.ob2);
  // dZ1 = (dZ2 W2) * [Z1 > 0]
  g = gemm(batch, H, H, w.dZ2b, H, 1, w.W2T, 1, H);
  g.mask = w.Z1;
  g.ldm = H;
  g.C32 = w.dZ1;
  g.ldc = H;
  if (tr) {
    g.C16T = w.dZ1T;
    g.ldt = batch;
  } else {
    g.C16 = w.dZ1b;
    g.ldc16 = H;
  }
  launch_gemm(g, st);
  // dW1 = dZ1^T X, db1
  g = tr ? gemm(H, F, batch, w.dZ1T, batch, 1, w.XT, 1, batch)
         : gemm(H, F, batch, w.dZ1b, 1, H, X, F, 1);
  g.C32 = grad + d.oW1;
  g.ldc = F;
  g.kpart = w.kpart;
  launch_gemm(g, st);
  cs.add(H, w.dZ1, grad + d.ob1);
  cs.launch(batch, w.part, st);
  CHECK_LAUNCH();
  return SCH_OK;
}

int sch_mlp_adam(const sch_mlp* net, const float* grad, float* m, float* v, int32_t step,
                 float lr, float beta1, float beta2, float eps, void* stream) {
  if (!mlp_ok(net) || !grad || !m || !v || step < 1 || !(lr > 0) || !(beta1 >= 0 && beta1 < 1) ||
      !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
    return fail(SCH_E_ARG, "bad arguments to sch_mlp_adam");
  const MlpDims d = mlp_dims(net->n_in, net->n_hidden, net->n_out);
  const float c1 = static_cast<float>(1.0 / (1.0 - std::pow(static_cast<double>(beta1), step)));
  const float c2 = static_cast<float>(1.0 / (1.0 - std::pow(static_cast<double>(beta2), step)));
  hipLaunchKernelGGL(k_adam, dim3(grid_for(d.n_params, 256)), dim3(256), 0, S(stream), d,
                     net->params, grad, m, v, lr, beta1, beta2, eps, c1, c2, net->weights_bf16);
  CHECK_LAUNCH();
  return SCH_OK;
}

int sch_mlp_features(const sch_model* md, const sch_obs* ob, int32_t n, const double* u,
                     const float* mean, const float* sdev, uint16_t* X, float* raw,
                     double* misfit, void* stream) {
  if (!md || md->nx < 2 || !ob || ob->n_obs < 1 || !ob->y || n < 1 || !u ||
      (X && (!mean || !sdev)) || (!X && !raw && !misfit))
    return fail(SCH_E_ARG, "bad arguments to sch_mlp_features");
  hipLaunchKernelGGL(k_mlp_features, dim3(n), dim3(256), 0, S(stream), md->nx, ob->n_obs, u,
                     ob->y, mean, sdev, X, raw, misfit);
  CHECK_LAUNCH();
  return SCH_OK;
}

int sch_mlp_colstats(int32_t rows, int32_t cols, const float* A, float* mean, float* sdev,
                     void* stream) {
  if (rows < 1 || cols < 1 || !A || !mean || !sdev)
    return fail(SCH_E_ARG, "bad arguments to sch_mlp_colstats");
  hipLaunchKernelGGL(k_colstats, dim3((cols + 255) / 256), dim3(256), 0, S(stream), rows, cols,
                     A, mean, sdev);
  CHECK_LAUNCH();
  return SCH_OK;
}

int sch_mlp_encode(int32_t n, int32_t cols, const float* raw, const float* mean,
                   const float* sdev, uint16_t* X, void* stream) {
  if (n < 1 || cols < 1 || !raw || !mean || !sdev || !X)
    return fail(SCH_E_ARG, "bad arguments to sch_mlp_encode");
  const int64_t total = static_cast<int64_t>(n) * cols;
  hipLaunchKernelGGL(k_mlp_encode, dim3(grid_for(total, 256)), dim3(256), 0, S(stream), total,
                     cols, raw, mean, sdev, X);
  CHECK_LAUNCH();
  return SCH_OK;
}

int sch_mlp_targets(int32_t n, int32_t cols, const double* dLam, const float* mean,
                    const float* sdev, float* T, void* stream) {
  if (n < 1 || cols < 1 || !dLam || !T || (mean && !sdev))
    return fail(SCH_E_ARG, "bad arguments to sch_mlp_targets");
  const int64_t total = static_cast<int64_t>(n) * cols;
  hipLaunchKernelGGL(k_mlp_targets, dim3(grid_for(total, 256)), dim3(256), 0, S(stream), total,
                     cols, dLam, mean, sdev, T);
  CHECK_LAUNCH();
  return SCH_OK;
}

int sch_mlp_controls(int32_t n, int32_t cols, const float* Y, const float* mean,
                     const float* sdev, const double* misfit, double threshold, double* dLam,
                     int32_t* mode, int32_t keep_mode, void* stream) {
  if (n < 1 || cols < 1 || !Y || !mean || !sdev || !dLam ||
      (mode && keep_mode != SCH_NUDGE_KEEP && keep_mode != SCH_NUDGE_FROM_GIVEN))
    return fail(SCH_E_ARG, "bad arguments to sch_mlp_controls");
  const int64_t total = static_cast<int64_t>(n) * cols;
  hipLaunchKernelGGL(k_mlp_controls, dim3(grid_for(total, 256)), dim3(256), 0, S(stream), total,
                     cols, Y, mean, sdev, misfit, threshold, dLam, mode, keep_mode,
                     SCH_NUDGE_FROM_ZERO);
  CHECK_LAUNCH();
  return SCH_OK;
}

}  // extern "C"
