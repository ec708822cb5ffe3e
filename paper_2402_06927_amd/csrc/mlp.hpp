// mlp.hpp -- kernels of the learned nudging warm start: a perceptron
// n_in -> H -> H -> n_out with ReLU, trained by mean-squared error and Adam.
// Matrix products run on the gfx950 matrix cores (v_mfma_f32_16x16x16bf16_1k:
// bfloat16 operands, float32 accumulation); weights keep a float32 master
// copy that Adam updates and a bfloat16 copy the products read.
//
// Parameter vector (float32): W1 [H][F], b1 [H], W2 [H][H], b2 [H],
// W3 [O][H], b3 [O]; the bfloat16 copy holds W1 | W2 | W3 back to back.
#pragma once

#include "device.hpp"

namespace sch {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// float32 -> bfloat16 bits, round to nearest, ties to even (NaN kept quiet).
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return static_cast<uint16_t>((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) {
  return __uint_as_float(static_cast<uint32_t>(b) << 16);
}

// C(m, n) = sum_k A(m, k) B(k, n) with A(m, k) = A[m sam + k sak] and
// B(k, n) = B[k sbk + n sbn] (one of the two strides of each operand is 1).
// Epilogue: v = C + bias[n]; v = 0 where mask[m][n] <= 0; C32 receives v,
// C16 receives bf16(relu ? max(v, 0) : v).
struct GemmArgs {
  int M, N, K;
  const uint16_t* A;
  int64_t sam, sak;
  const uint16_t* B;
  int64_t sbk, sbn;
  float* C32;
  int64_t ldc;
  uint16_t* C16;
  int64_t ldc16;
  const float* bias;
  const float* mask;
  int64_t ldm;
  int relu;
};

constexpr int kGM = 64, kGN = 64, kGK = 32, kGPad = 8;  // LDS rows of 80 bytes

// Epilogue and matrix-core steps shared by both loaders.
__device__ __forceinline__ void gemm_chunk(const uint16_t (&As)[kGM][kGK + kGPad],
                                           const uint16_t (&Bs)[kGN][kGK + kGPad], int wm,
                                           int wn, int lane, f32x4 (&acc)[2][2]) {
#pragma unroll
  for (int ks = 0; ks < kGK; ks += 16) {
    bf16x4 a[2], b[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      a[i] = *reinterpret_cast<const bf16x4*>(&As[wm + 16 * i + (lane & 15)][ks + 4 * (lane >> 4)]);
      b[i] = *reinterpret_cast<const bf16x4*>(&Bs[wn + 16 * i + (lane & 15)][ks + 4 * (lane >> 4)]);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[i], b[j], acc[i][j], 0, 0, 0);
  }
}

__device__ __forceinline__ void gemm_store(const GemmArgs& g, int m0, int n0, int wm, int wn,
                                           int lane, const f32x4 (&acc)[2][2]) {
  // lane l of a 16 x 16 tile holds rows 4 (l / 16) .. + 3 of column l % 16
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm + 16 * i + 4 * (lane >> 4) + r;
        const int n = n0 + wn + 16 * j + (lane & 15);
        if (m >= g.M || n >= g.N) continue;
        float v = acc[i][j][r];
        if (g.bias) v += g.bias[n];
        if (g.mask && !(g.mask[m * g.ldm + n] > 0.f)) v = 0.f;
        if (g.C32) g.C32[m * g.ldc + n] = v;
        if (g.C16) g.C16[m * g.ldc16 + n] = f2bf(g.relu ? fmaxf(v, 0.f) : v);
      }
}

// 256 threads = 4 wavefronts, each computing a 32 x 32 block as 2 x 2 matrix-
// core tiles of 16 x 16; K advances in chunks of 32 staged in LDS.  Element-
// wise loads: any operand layout with one unit stride.
__global__ void __launch_bounds__(256) k_gemm_bf16(const GemmArgs g) {
  __shared__ __attribute__((aligned(16))) uint16_t As[kGM][kGK + kGPad];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[kGN][kGK + kGPad];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int m0 = blockIdx.y * kGM, n0 = blockIdx.x * kGN;
  const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const bool a_kfast = g.sak == 1, b_kfast = g.sbk == 1;
  for (int k0 = 0; k0 < g.K; k0 += kGK) {
#pragma unroll
    for (int i = 0; i < (kGM * kGK) / 256; ++i) {
      const int e = t + 256 * i;
      const int mm = a_kfast ? e / kGK : e % kGM, kk = a_kfast ? e % kGK : e / kGM;
      const int gm = m0 + mm, gk = k0 + kk;
      As[mm][kk] = (gm < g.M && gk < g.K) ? g.A[gm * g.sam + gk * g.sak] : uint16_t(0);
      const int nn = b_kfast ? e / kGK : e % kGN, kb = b_kfast ? e % kGK : e / kGN;
      const int gn = n0 + nn, gkb = k0 + kb;
      Bs[nn][kb] = (gn < g.N && gkb < g.K) ? g.B[gkb * g.sbk + gn * g.sbn] : uint16_t(0);
    }
    __syncthreads();
    gemm_chunk(As, Bs, wm, wn, lane, acc);
    __syncthreads();
  }
  gemm_store(g, m0, n0, wm, wn, lane, acc);
}

// Both operands contiguous along K (sak = sbk = 1), K, sam, sbn multiples of 8
// and 16-byte aligned rows: each thread moves 8 bf16 of A and of B per chunk
// with one 16-byte load each, and the next chunk is fetched into registers
// while the matrix cores work on the current one.
__global__ void __launch_bounds__(256) k_gemm_bf16_kc(const GemmArgs g) {
  __shared__ __attribute__((aligned(16))) uint16_t As[kGM][kGK + kGPad];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[kGN][kGK + kGPad];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int m0 = blockIdx.y * kGM, n0 = blockIdx.x * kGN;
  const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
  const int row = t >> 2, seg = (t & 3) * 8;  // 64 rows x 4 segments of 8
  const int gm = m0 + row, gn = n0 + row;
  const uint4 zero = make_uint4(0u, 0u, 0u, 0u);
  // a segment is read only when it lies inside the row (k0 + seg < K implies
  // k0 + seg + 8 <= K since both are multiples of 8)
  auto fetch = [&](int k0, uint4& ra, uint4& rb) {
    const bool in_k = k0 + seg < g.K;
    ra = (gm < g.M && in_k) ? *reinterpret_cast<const uint4*>(g.A + gm * g.sam + k0 + seg) : zero;
    rb = (gn < g.N && in_k) ? *reinterpret_cast<const uint4*>(g.B + gn * g.sbn + k0 + seg) : zero;
  };
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  uint4 ra, rb;
  fetch(0, ra, rb);
  for (int k0 = 0; k0 < g.K; k0 += kGK) {
    // K is a multiple of 8 but maybe not of 32: zero the segments past K
    if (k0 + seg >= g.K) {
      ra = zero;
      rb = zero;
    }
    *reinterpret_cast<uint4*>(&As[row][seg]) = ra;
    *reinterpret_cast<uint4*>(&Bs[row][seg]) = rb;
    __syncthreads();
    if (k0 + kGK < g.K) fetch(k0 + kGK, ra, rb);
    gemm_chunk(As, Bs, wm, wn, lane, acc);
    __syncthreads();
  }
  gemm_store(g, m0, n0, wm, wn, lane, acc);
}

// Mean-squared error of Y against T ([rows][cols]) and its gradient
// dY = 2 (Y - T) / (rows cols) (float32 and bfloat16); *loss accumulates.
__global__ void k_mse(int64_t n, const float* Y, const float* T, float inv_count, float* dY32,
                      uint16_t* dY16, double* loss) {
  double acc = 0.0;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const float r = Y[i] - T[i];
    const float d = 2.0f * r * inv_count;
    dY32[i] = d;
    dY16[i] = f2bf(d);
    acc += static_cast<double>(r) * r;
  }
  // one atomic per workgroup (blockDim.x = 256): per-wavefront atomics on the
  // one address serialise
  __shared__ double part[4];
  acc = wave_sum(acc);
  if ((threadIdx.x & (kWave - 1)) == 0) part[threadIdx.x / kWave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(loss, ((part[0] + part[1]) + (part[2] + part[3])) * inv_count);
}

// Column sums out[c] = sum_r A[r][c] in two passes with a fixed order.
// Pass 1 (grid (ceil(cols / 64), ceil(rows / kColsumRows)), 256 threads):
// workgroup (x, b) sums the rows of slice b for 64 columns, 4 row lanes each
// taking every 4th row in float64, the lanes combined in lane order, into
// part[b][c].  Pass 2 adds the slices' partials in slice order.  Every
// workgroup's share is short, so the sums are spread over the whole chip.
constexpr int kColsumRows = 64;

__global__ void __launch_bounds__(256) k_colsum_part(int rows, int cols, const float* A,
                                                     double* part) {
  __shared__ double red[4][64];
  const int cl = threadIdx.x & 63, rl = threadIdx.x >> 6;
  const int c = blockIdx.x * 64 + cl;
  const int r0 = blockIdx.y * kColsumRows, r1 = min(rows, r0 + kColsumRows);
  double s = 0.0;
  if (c < cols)
    for (int r = r0 + rl; r < r1; r += 4) s += A[static_cast<int64_t>(r) * cols + c];
  red[rl][cl] = s;
  __syncthreads();
  if (rl == 0 && c < cols)
    part[static_cast<int64_t>(blockIdx.y) * cols + c] =
        ((red[0][cl] + red[1][cl]) + red[2][cl]) + red[3][cl];
}

__global__ void k_colsum_final(int n_part, int cols, const double* part, float* out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  double t = 0.0;
  for (int b = 0; b < n_part; ++b) t += part[static_cast<int64_t>(b) * cols + c];
  out[c] = static_cast<float>(t);
}

// out[c][r] = in[r][c] for a rows x cols bfloat16 matrix (leading dimensions
// ldi, ldo), through LDS in 64 x 64 tiles: both the reads and the writes
// move consecutive elements across consecutive threads.
__global__ void __launch_bounds__(256) k_transpose_bf16(int rows, int cols, const uint16_t* in,
                                                        int64_t ldi, uint16_t* out, int64_t ldo) {
  __shared__ uint16_t tile[64][66];
  const int c0 = blockIdx.x * 64, r0 = blockIdx.y * 64;
  for (int i = threadIdx.x; i < 64 * 64; i += 256) {
    const int r = i >> 6, c = i & 63;
    const int gr = r0 + r, gc = c0 + c;
    tile[r][c] = (gr < rows && gc < cols) ? in[gr * ldi + gc] : uint16_t(0);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 64 * 64; i += 256) {
    const int c = i >> 6, r = i & 63;
    const int gr = r0 + r, gc = c0 + c;
    if (gr < rows && gc < cols) out[gc * ldo + gr] = tile[r][c];
  }
}

// Column means and standard deviations (two passes, float64 accumulation);
// a column whose deviation is below 1e-12 gets deviation 1.
__global__ void k_colstats(int rows, int cols, const float* A, float* mean, float* sdev) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  double s = 0.0;
  for (int r = 0; r < rows; ++r) s += A[static_cast<int64_t>(r) * cols + c];
  const double mu = s / rows;
  double q = 0.0;
  for (int r = 0; r < rows; ++r) {
    const double d = A[static_cast<int64_t>(r) * cols + c] - mu;
    q += d * d;
  }
  const double sd = sqrt(q / rows);
  mean[c] = static_cast<float>(mu);
  sdev[c] = sd > 1e-12 ? static_cast<float>(sd) : 1.0f;
}

struct MlpDims {
  int F, H, O;
  int64_t oW1, ob1, oW2, ob2, oW3, ob3, n_params;  // offsets in the parameter vector
  int64_t qW2, qW3, n_weights;                     // offsets in the bfloat16 copy
};

__host__ __device__ inline MlpDims mlp_dims(int F, int H, int O) {
  MlpDims d;
  d.F = F;
  d.H = H;
  d.O = O;
  d.oW1 = 0;
  d.ob1 = d.oW1 + static_cast<int64_t>(H) * F;
  d.oW2 = d.ob1 + H;
  d.ob2 = d.oW2 + static_cast<int64_t>(H) * H;
  d.oW3 = d.ob2 + H;
  d.ob3 = d.oW3 + static_cast<int64_t>(O) * H;
  d.n_params = d.ob3 + O;
  d.qW2 = static_cast<int64_t>(H) * F;
  d.qW3 = d.qW2 + static_cast<int64_t>(H) * H;
  d.n_weights = d.qW3 + static_cast<int64_t>(O) * H;
  return d;
}

// Position of parameter i in the bfloat16 weight copy, or -1 for a bias.
__device__ __forceinline__ int64_t weight_slot(const MlpDims& d, int64_t i) {
  if (i < d.ob1) return i;
  if (i >= d.oW2 && i < d.ob2) return d.qW2 + (i - d.oW2);
  if (i >= d.oW3 && i < d.ob3) return d.qW3 + (i - d.oW3);
  return -1;
}

// Adam (Kingma & Ba, Algorithm 1) on the float32 master copy, bias
// corrections c1 = 1 / (1 - beta1^t), c2 = 1 / (1 - beta2^t) given by the
// caller; refreshes the bfloat16 weight copy.  With grad == nullptr only the
// copy is refreshed.
__global__ void k_adam(MlpDims d, float* p, const float* grad, float* m, float* v, float lr,
                       float beta1, float beta2, float eps, float c1, float c2, uint16_t* wb) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < d.n_params;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    float w = p[i];
    if (grad) {
      const float gi = grad[i];
      const float mi = beta1 * m[i] + (1.0f - beta1) * gi;
      const float vi = beta2 * v[i] + (1.0f - beta2) * gi * gi;
      m[i] = mi;
      v[i] = vi;
      w -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
      p[i] = w;
    }
    const int64_t q = weight_slot(d, i);
    if (q >= 0) wb[q] = f2bf(w);
  }
}

// Network inputs of one particle (reading of the input description):
// the observation misfit y - P u (n_obs values) followed by the velocity u
// (nx values), standardised with the training means and deviations and
// rounded to bfloat16.  raw (float32, optional) receives the unscaled values,
// misfit (optional) the Euclidean norm of y - P u.  One workgroup per particle.
__global__ void k_mlp_features(int nx, int n_obs, const double* u, const double* y,
                               const float* mean, const float* sdev, uint16_t* X, float* raw,
                               double* misfit) {
  const int p = blockIdx.x, F = n_obs + nx;
  const double* up = u + static_cast<int64_t>(p) * nx;
  __shared__ double red[16];
  double acc = 0.0;
  for (int j = threadIdx.x; j < F; j += blockDim.x) {
    double x;
    if (j < n_obs) {
      const int64_t num = static_cast<int64_t>(j) * nx;
      const int e = static_cast<int>(num / n_obs);
      const double r = static_cast<double>(num % n_obs) / static_cast<double>(n_obs);
      const int e1 = e + 1 == nx ? 0 : e + 1;
      x = y[j] - ((1.0 - r) * up[e] + r * up[e1]);
      acc += x * x;
    } else {
      x = up[j - n_obs];
    }
    const int64_t o = static_cast<int64_t>(p) * F + j;
    if (raw) raw[o] = static_cast<float>(x);
    if (X) X[o] = f2bf((static_cast<float>(x) - mean[j]) / sdev[j]);
  }
  acc = wave_sum(acc);
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = acc;
  __syncthreads();
  if (threadIdx.x == 0 && misfit) {
    double s = 0.0;
    for (int i = 0; i < static_cast<int>(blockDim.x) / kWave; ++i) s += red[i];
    misfit[p] = sqrt(s);
  }
}

// Stored raw features to network inputs: X = bf16((raw - mean) / sdev), the
// same arithmetic as the scaling path of k_mlp_features.
__global__ void k_mlp_encode(int64_t n, int cols, const float* raw, const float* mean,
                             const float* sdev, uint16_t* X) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int c = static_cast<int>(i % cols);
    X[i] = f2bf((raw[i] - mean[c]) / sdev[c]);
  }
}

// Training targets: T = (dLambda - mean) / sdev in float32 (raw float32 copy
// of dLambda in `raw` when mean is null).
__global__ void k_mlp_targets(int64_t n, int cols, const double* dLam, const float* mean,
                              const float* sdev, float* out) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const float x = static_cast<float>(dLam[i]);
    const int c = static_cast<int>(i % cols);
    out[i] = mean ? (x - mean[c]) / sdev[c] : x;
  }
}

// Warm start from the network output: dLambda = Y sdev + mean, or zero (the
// plain start) for particles whose misfit norm exceeds the threshold.
// mode (optional): per particle, keep_mode where the prediction is used and
// fallback_mode where the misfit is above the threshold (the start modes of
// sch_pf_nudged_cycle_warm).
__global__ void k_mlp_controls(int64_t n, int cols, const float* Y, const float* mean,
                               const float* sdev, const double* misfit, double threshold,
                               double* dLam, int* mode, int keep_mode, int fallback_mode) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int c = static_cast<int>(i % cols);
    const int64_t p = i / cols;
    const bool plain = misfit && !(misfit[p] <= threshold);
    dLam[i] = plain ? 0.0 : static_cast<double>(Y[i] * sdev[c] + mean[c]);
    if (mode && c == 0) mode[p] = plain ? fallback_mode : keep_mode;
  }
}

}  // namespace sch
