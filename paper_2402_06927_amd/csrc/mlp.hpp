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
// C16 receives bf16(relu ? max(v, 0) : v) and C16T the same value transposed
// (C16T[n ldt + m]; ldt a multiple of 4 and C16T 8-byte aligned).
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
  uint16_t* C16T;
  int64_t ldt;
  const float* bias;
  const float* mask;
  int64_t ldm;
  int relu;
  float* kpart;  // split-K partial products [gridDim.z][M][N] (K-contiguous loaders), or null
};

constexpr int kGM = 64, kGN = 64, kGK = 32, kGPad = 8;  // LDS rows of 80 bytes

// Epilogue and matrix-core steps shared by both loaders: a chunk of KC
// values of k in steps of 16 (the sums run over k in the same order for any
// chunk width).
template <int KC>
__device__ __forceinline__ void gemm_chunk(const uint16_t (&As)[kGM][KC + kGPad],
                                           const uint16_t (&Bs)[kGN][KC + kGPad], int wm,
                                           int wn, int lane, f32x4 (&acc)[2][2]) {
#pragma unroll
  for (int ks = 0; ks < KC; ks += 16) {
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

// Epilogue of one element of C; returns its bf16 value. TP: write the
// transposed copy here (the tiled stores write it four rows at a time).
template <bool TP = true>
__device__ __forceinline__ uint16_t gemm_epilogue(const GemmArgs& g, int m, int n, float v) {
  if (g.bias) v += g.bias[n];
  if (g.mask && !(g.mask[m * g.ldm + n] > 0.f)) v = 0.f;
  if (g.C32) g.C32[m * g.ldc + n] = v;
  const uint16_t b = f2bf(g.relu ? fmaxf(v, 0.f) : v);
  if (g.C16) g.C16[m * g.ldc16 + n] = b;
  if (TP && g.C16T) g.C16T[n * g.ldt + m] = b;
  return b;
}

// RAW: the accumulators go to the split-K partials of slice `z` instead.
template <bool RAW = false>
__device__ __forceinline__ void gemm_store(const GemmArgs& g, int m0, int n0, int wm, int wn,
                                           int lane, const f32x4 (&acc)[2][2], int z = 0) {
  // lane l of a 16 x 16 tile holds rows 4 (l / 16) .. + 3 of column l % 16
  if (!RAW && g.C16T) {
    // m0, wm are multiples of 16: the four rows start at a multiple of 4 and
    // land in one 8-byte word of the transposed copy
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int m = m0 + wm + 16 * i + 4 * (lane >> 4);
        const int n = n0 + wn + 16 * j + (lane & 15);
        if (n >= g.N) continue;
        if (m + 3 < g.M) {
          uint16_t b[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) b[r] = gemm_epilogue<false>(g, m + r, n, acc[i][j][r]);
          *reinterpret_cast<uint2*>(g.C16T + n * g.ldt + m) =
              make_uint2(b[0] | (static_cast<uint32_t>(b[1]) << 16),
                         b[2] | (static_cast<uint32_t>(b[3]) << 16));
        } else {
          for (int r = 0; r < 4 && m + r < g.M; ++r) gemm_epilogue(g, m + r, n, acc[i][j][r]);
        }
      }
    return;
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm + 16 * i + 4 * (lane >> 4) + r;
        const int n = n0 + wn + 16 * j + (lane & 15);
        if (m >= g.M || n >= g.N) continue;
        if constexpr (RAW)
          g.kpart[(static_cast<int64_t>(z) * g.M + m) * g.N + n] = acc[i][j][r];
        else
          gemm_epilogue(g, m, n, acc[i][j][r]);
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
    gemm_chunk<kGK>(As, Bs, wm, wn, lane, acc);
    __syncthreads();
  }
  gemm_store(g, m0, n0, wm, wn, lane, acc);
}

// Both operands contiguous along K (sak = sbk = 1), K, sam, sbn multiples of 8
// and 16-byte aligned rows.  K advances in chunks of KC staged in LDS, each
// thread moving KC / 32 segments of 8 bf16 of A and of B per chunk with
// 16-byte loads (a wavefront's load covers 256 / KC * 4 rows of whole
// 2 KC-byte spans).  With one workgroup per compute unit (the large products
// have only about as many tiles as the chip has units) every chunk pays a
// serial chain of LDS stores, a barrier, LDS reads and dependent matrix-core
// steps, so the chunks are wide (128 values of k), the LDS tile is double
// buffered (one barrier per chunk) and DEPTH chunks are loaded ahead into
// registers.  Tile order: consecutive workgroups go to different XCDs
// (round-robin), each with its own L2; the tiles are renumbered so that the
// column tiles of one row block run on the same XCD and read that block of A
// through one L2.  The sums are those of k_gemm_bf16, in the same order.
// Split K as in k_gemm_bf16_lds (below), in whole chunks of KC.
template <int KC, int DEPTH>
__global__ void __launch_bounds__(256) k_gemm_bf16_kc(const GemmArgs g) {
  static_assert(DEPTH % 2 == 0, "the LDS buffer of a stage is fixed");
  static_assert(KC % 32 == 0 && KC <= 128, "chunk of whole 32-value passes");
  constexpr int SEGS = KC / 8, PASS = KC / 32, RSTEP = 256 / SEGS;
  __shared__ __attribute__((aligned(16))) uint16_t As[2][kGM][KC + kGPad];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[2][kGN][KC + kGPad];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int nbx = gridDim.x, ntile = gridDim.x * gridDim.y;
  int tile = blockIdx.y * nbx + blockIdx.x;
  if (ntile % 8 == 0) tile = (tile % 8) * (ntile / 8) + tile / 8;
  const int m0 = (tile / nbx) * kGM, n0 = (tile % nbx) * kGN;
  const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
  const int row0 = t / SEGS, seg = (t % SEGS) * 8;  // rows row0 + RSTEP i
  // split K (gridDim.z > 1, K a multiple of KC): slice z takes the chunks
  // c_lo .. c_hi - 1 of KC values and stores raw partial sums
  const int nz = gridDim.z, z = blockIdx.z;
  const int c_lo = nz > 1 ? z * (g.K / KC) / nz : 0;
  const int kl = nz > 1 ? ((z + 1) * (g.K / KC) / nz - c_lo) * KC : g.K;
  // Loads are never predicated (a branch around them would make the compiler
  // wait for every load in flight before the next LDS store): rows past M or
  // N and segments past K read the last valid row or segment, and the value
  // is replaced by zero.  Segments start at multiples of 8 and K is one, so a
  // segment lies inside the row or wholly past K.
  const uint16_t* pa[PASS];
  const uint16_t* pb[PASS];
  bool arow[PASS], brow[PASS];
#pragma unroll
  for (int i = 0; i < PASS; ++i) {
    const int gm = m0 + row0 + RSTEP * i, gn = n0 + row0 + RSTEP * i;
    pa[i] = g.A + static_cast<int64_t>(min(gm, g.M - 1)) * g.sam + c_lo * KC;
    pb[i] = g.B + static_cast<int64_t>(min(gn, g.N - 1)) * g.sbn + c_lo * KC;
    arow[i] = gm < g.M;
    brow[i] = gn < g.N;
  }
  auto ld = [&](const uint16_t* p, bool ok, int k0) -> uint4 {
    const int k = k0 + seg;
    uint4 v = *reinterpret_cast<const uint4*>(p + min(k, kl - 8));
    ok = ok && k < kl;
    v.x = ok ? v.x : 0u;
    v.y = ok ? v.y : 0u;
    v.z = ok ? v.z : 0u;
    v.w = ok ? v.w : 0u;
    return v;
  };
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  // the chunk count is rounded up to a multiple of DEPTH: the chunks past K
  // are zero and add exact zeros
  const int nk = (kl + KC - 1) / KC;
  uint4 ra[DEPTH][PASS], rb[DEPTH][PASS];
#pragma unroll
  for (int s = 0; s < DEPTH; ++s)
#pragma unroll
    for (int i = 0; i < PASS; ++i) {
      ra[s][i] = ld(pa[i], arow[i], s * KC);
      rb[s][i] = ld(pb[i], brow[i], s * KC);
    }
  for (int c0 = 0; c0 < nk; c0 += DEPTH) {
#pragma unroll
    for (int s = 0; s < DEPTH; ++s) {
      const int c = c0 + s, b = s & 1;  // DEPTH is even: buffer c % 2
#pragma unroll
      for (int i = 0; i < PASS; ++i) {
        *reinterpret_cast<uint4*>(&As[b][row0 + RSTEP * i][seg]) = ra[s][i];
        *reinterpret_cast<uint4*>(&Bs[b][row0 + RSTEP * i][seg]) = rb[s][i];
      }
      // every wavefront has finished chunk c - 1 (which read the other
      // buffer) before any passes this barrier, and chunk c - 2 (which read
      // this one) before it stored chunk c - 1
      __syncthreads();
#pragma unroll
      for (int i = 0; i < PASS; ++i) {
        ra[s][i] = ld(pa[i], arow[i], (c + DEPTH) * KC);
        rb[s][i] = ld(pb[i], brow[i], (c + DEPTH) * KC);
      }
      gemm_chunk<KC>(As[b], Bs[b], wm, wn, lane, acc);
    }
  }
  if (nz > 1)
    gemm_store<true>(g, m0, n0, wm, wn, lane, acc, z);
  else
    gemm_store(g, m0, n0, wm, wn, lane, acc);
}

// Output tiles of TM x TM (64 or 128).  Operands contiguous along K with K a
// multiple of kLC, sam, sbn multiples of 8 and 16-byte aligned rows.  The
// operands travel from global memory to LDS without registers
// (global_load_lds_dwordx4): one instruction moves a block of 16 rows x 32
// values of k, lane l taking row l % 16 and values 8 (l / 16) .. + 7, and
// lands it in LDS in lane order, which is the layout in which the
// 16 x 16 x 32 bf16 matrix instruction takes its operands (lane l: row
// l % 16, the same eight values of k for A and B), so each operand is read
// back with one conflict-free 16-byte LDS read per lane.  A stage holds 16
// blocks of each operand: TM / 16 row blocks by KC / 32 blocks of k, so a
// chunk is KC = 512 / (TM / 16) values of k (128 for 64-row tiles, 64 for
// 128-row ones).  A ring of kLS stages (32 KB each) keeps kLS - 1 chunks in
// flight per compute unit, as the products are bound by the rate at which
// their loads arrive; one barrier per chunk.  Each wavefront computes a
// (TM / 2) x (TM / 2) quarter of the tile.  Rows past M or N read the last
// row (their results are not stored).  Tile order as in k_gemm_bf16_kc.
// Within a chunk the sums run over k in steps of 32.  The 128-row tile moves
// half the bytes per product of the 64-row one (each unit's loads are the
// bound: about 30 GB/s per unit from L2).
// Split K (gridDim.z > 1, when the tiles alone would leave compute units
// idle): slice z takes chunks [z nk / Z, (z + 1) nk / Z) and writes its raw
// sums to g.kpart; k_gemm_reduce adds the slices in order and applies the
// epilogue.
constexpr int kLC = 128, kLS = 4;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  // s_waitcnt with vmcnt = N (bits 3:0 and 15:14), expcnt and lgkmcnt at
  // their maxima (no wait)
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}

// 16 bytes per lane from global memory straight to LDS, in lane order from
// the wavefront's base address lds
__device__ __forceinline__ void load_lds16(const uint16_t* p, uint4* lds) {
  __builtin_amdgcn_global_load_lds(p, lds, 16, 0, 0);
}

template <int TM>
__global__ void __launch_bounds__(256) k_gemm_bf16_lds(const GemmArgs g) {
  static_assert(TM == 64 || TM == 128, "tile edge");
  // RB row blocks of 16 by QB blocks of 32 values of k per operand and stage;
  // each wavefront loads RPW row blocks, and computes WB x WB matrix-core tiles
  constexpr int RB = TM / 16, QB = 16 / RB, KC = 32 * QB, RPW = RB / 4, WB = TM / 32;
  static_assert(2 * RPW * QB == 8, "eight loads per wavefront and chunk (the waits below)");
  // [stage][operand][block = row block x QB + k block][lane]
  __shared__ __attribute__((aligned(16))) uint4 T[kLS][2][16][64];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int nbx = gridDim.x, ntile = gridDim.x * gridDim.y;
  int tile = blockIdx.y * nbx + blockIdx.x;
  if (ntile % 8 == 0) tile = (tile % 8) * (ntile / 8) + tile / 8;
  const int m0 = (tile / nbx) * TM, n0 = (tile % nbx) * TM;
  // an LDS store the compiler can see (never taken for valid sizes): without
  // one it takes the array for never written and drops the reads
  if (g.M <= 0) T[0][0][0][lane] = make_uint4(0u, 0u, 0u, 0u);
  // wave w loads row blocks RPW w .. + RPW - 1 of A and of B: lane l of block
  // (rb, q) reads row 16 rb + l % 16 at k = 32 q + 8 (l / 16)
  const int kl = 8 * (lane >> 4);
  const int nk_all = g.K / KC, nz = gridDim.z, z = blockIdx.z;
  const int c_lo = (nk_all * z) / nz, nk = (nk_all * (z + 1)) / nz - c_lo;
  const uint16_t* pa[RPW];
  const uint16_t* pb[RPW];
#pragma unroll
  for (int i = 0; i < RPW; ++i) {
    const int r = 16 * (RPW * w + i) + (lane & 15);
    pa[i] = g.A + static_cast<int64_t>(min(m0 + r, g.M - 1)) * g.sam + kl +
            static_cast<int64_t>(c_lo) * KC;
    pb[i] = g.B + static_cast<int64_t>(min(n0 + r, g.N - 1)) * g.sbn + kl +
            static_cast<int64_t>(c_lo) * KC;
  }
  auto issue = [&](int c, int st) {
    const int k0 = c * KC;
#pragma unroll
    for (int i = 0; i < RPW; ++i)
#pragma unroll
      for (int q = 0; q < QB; ++q) {
        const int b = (RPW * w + i) * QB + q;
        load_lds16(pa[i] + k0 + 32 * q, &T[st][0][b][0]);
        load_lds16(pb[i] + k0 + 32 * q, &T[st][1][b][0]);
      }
  };
  const int wm = (w >> 1) * WB, wn = (w & 1) * WB;  // this wave's first row and column blocks
  f32x4 acc[WB][WB];
#pragma unroll
  for (int i = 0; i < WB; ++i)
#pragma unroll
    for (int j = 0; j < WB; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int c = 0; c < kLS - 1; ++c)
    if (c < nk) issue(c, c);
  for (int c = 0; c < nk; ++c) {
    // this wave's loads of chunk c are done once at most those of the chunks
    // issued after it (8 instructions each) are outstanding
    const int after = min(kLS - 2, nk - 1 - c);
    if (after >= 2)
      wait_vmcnt<16>();
    else if (after == 1)
      wait_vmcnt<8>();
    else
      wait_vmcnt<0>();
    // every wavefront's part of chunk c is in LDS, and every wavefront has
    // finished chunk c - 1, whose stage is refilled next.  A plain barrier:
    // __syncthreads() would also wait for every load in flight (its fence),
    // and each wavefront has already waited for its own part of chunk c;
    // the LDS reads of chunk c - 1 completed before the matrix steps that
    // used them.  The empty asm with a memory clobber keeps the compiler from
    // moving LDS accesses across the barrier.
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    if (c + kLS - 1 < nk) issue(c + kLS - 1, (c + kLS - 1) % kLS);
    const int st = c % kLS;
#pragma unroll
    for (int q = 0; q < QB; ++q) {
      bf16x8 a[WB], b[WB];
#pragma unroll
      for (int i = 0; i < WB; ++i) {
        a[i] = *reinterpret_cast<const bf16x8*>(&T[st][0][(wm + i) * QB + q][lane]);
        b[i] = *reinterpret_cast<const bf16x8*>(&T[st][1][(wn + i) * QB + q][lane]);
      }
#pragma unroll
      for (int i = 0; i < WB; ++i)
#pragma unroll
        for (int j = 0; j < WB; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  }
  // the stores take 2 x 2 matrix-core tiles at a time
#pragma unroll
  for (int qi = 0; qi < WB; qi += 2)
#pragma unroll
    for (int qj = 0; qj < WB; qj += 2) {
      const f32x4 sub[2][2] = {{acc[qi][qj], acc[qi][qj + 1]}, {acc[qi + 1][qj], acc[qi + 1][qj + 1]}};
      if (nz > 1)
        gemm_store<true>(g, m0, n0, 16 * (wm + qi), 16 * (wn + qj), lane, sub, z);
      else
        gemm_store(g, m0, n0, 16 * (wm + qi), 16 * (wn + qj), lane, sub);
    }
}

// The sum of the nz split-K slices of a K-contiguous loader (in slice order), then
// the epilogue, one element per thread (consecutive elements across lanes, so
// the epilogue's stores coalesce).
__global__ void k_gemm_reduce(const GemmArgs g, int nz) {
  const int64_t mn = static_cast<int64_t>(g.M) * g.N;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < mn;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    float v = g.kpart[i];
    for (int z = 1; z < nz; ++z) v += g.kpart[z * mn + i];
    gemm_epilogue(g, static_cast<int>(i / g.N), static_cast<int>(i % g.N), v);
  }
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

// Column sums out_k[c] = sum_r A_k[r][c] of up to kColsumBatch float32
// matrices with the same number of rows, in two passes with a fixed order.
// Pass 1 (grid (total column tiles of 64, ceil(rows / kColsumRows)), 256
// threads): workgroup (x, b) sums the rows of slice b for 64 columns of one
// matrix (matrix k owns column tiles tile0[k] .. tile0[k + 1] - 1), 4 row
// lanes each taking every 4th row in float64, the lanes combined in lane
// order, into part[b][coff[k] + c].  Pass 2 adds the slices' partials in
// slice order.  Every workgroup's share is short, so the sums are spread
// over the whole chip.
constexpr int kColsumRows = 64, kColsumBatch = 4;
struct ColsumBatch {
  int n;
  int cols[kColsumBatch];
  int tile0[kColsumBatch + 1], coff[kColsumBatch + 1];
  const float* A[kColsumBatch];
  float* out[kColsumBatch];
};

__global__ void __launch_bounds__(256) k_colsum_part(int rows, const ColsumBatch b,
                                                     double* part) {
  __shared__ double red[4][64];
  int k = 0;
  while (k + 1 < b.n && static_cast<int>(blockIdx.x) >= b.tile0[k + 1]) ++k;
  const int cl = threadIdx.x & 63, rl = threadIdx.x >> 6;
  const int c = (blockIdx.x - b.tile0[k]) * 64 + cl, cols = b.cols[k];
  const float* A = b.A[k];
  const int r0 = blockIdx.y * kColsumRows, r1 = min(rows, r0 + kColsumRows);
  double s = 0.0;
  if (c < cols)
    for (int r = r0 + rl; r < r1; r += 4) s += A[static_cast<int64_t>(r) * cols + c];
  red[rl][cl] = s;
  __syncthreads();
  if (rl == 0 && c < cols)
    part[static_cast<int64_t>(blockIdx.y) * b.coff[b.n] + b.coff[k] + c] =
        ((red[0][cl] + red[1][cl]) + red[2][cl]) + red[3][cl];
}

__global__ void k_colsum_final(int n_part, const ColsumBatch b, const double* part) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x, ctot = b.coff[b.n];
  if (c >= ctot) return;
  int k = 0;
  while (k + 1 < b.n && c >= b.coff[k + 1]) ++k;
  double t = 0.0;
  for (int s = 0; s < n_part; ++s) t += part[static_cast<int64_t>(s) * ctot + c];
  b.out[k][c - b.coff[k]] = static_cast<float>(t);
}

// Up to kTransposeBatch independent transposes out[c][r] = in[r][c] of dense
// rows x cols bfloat16 matrices in one launch, through LDS in 64 x 64 tiles
// (both the reads and the writes move consecutive elements across
// consecutive threads): matrix i owns workgroups tile0[i] .. tile0[i + 1] - 1,
// its tiles numbered along the columns first (tx[i] tiles to a row of tiles).
constexpr int kTransposeBatch = 8;
struct TransposeBatch {
  int n;
  int rows[kTransposeBatch], cols[kTransposeBatch], tx[kTransposeBatch];
  int tile0[kTransposeBatch + 1];
  const uint16_t* in[kTransposeBatch];
  uint16_t* out[kTransposeBatch];
};

__global__ void __launch_bounds__(256) k_transpose_bf16(const TransposeBatch b) {
  __shared__ uint16_t tile[64][66];
  int k = 0;
  while (k + 1 < b.n && static_cast<int>(blockIdx.x) >= b.tile0[k + 1]) ++k;
  const int loc = blockIdx.x - b.tile0[k], rows = b.rows[k], cols = b.cols[k];
  const int r0 = (loc / b.tx[k]) * 64, c0 = (loc % b.tx[k]) * 64;
  const uint16_t* in = b.in[k];
  uint16_t* out = b.out[k];
  for (int i = threadIdx.x; i < 64 * 64; i += 256) {
    const int r = i >> 6, c = i & 63;
    const int gr = r0 + r, gc = c0 + c;
    tile[r][c] = (gr < rows && gc < cols) ? in[static_cast<int64_t>(gr) * cols + gc] : uint16_t(0);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 64 * 64; i += 256) {
    const int c = i >> 6, r = i & 63;
    const int gr = r0 + r, gc = c0 + c;
    if (gr < rows && gc < cols) out[static_cast<int64_t>(gc) * rows + gr] = tile[r][c];
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
