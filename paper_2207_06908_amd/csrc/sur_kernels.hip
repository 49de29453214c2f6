// sur_kernels.hip -- kernels of the surrogate network on gfx950.
//
// Products are C = A B^T with both operands bfloat16 and K-contiguous, on
// the CDNA4 matrix cores (v_mfma_f32_16x16x32_bf16, FP32 accumulation).  The
// producers of every operand write it in the layout its consumer wants: the
// forward epilogue writes each activation both row-major (input of the next
// layer) and transposed (input of the weight-gradient product), the backward
// epilogue does the same for the output-side gradient, and Adam keeps W and
// W^T copies.  So every product reads 16-byte vectors along K and no kernel
// transposes through LDS.
//
// Fragment layout of the 16x16x32 instruction (64 lanes): lane l supplies
// A[row l%16][k = 8(l/16) .. 8(l/16)+7] and B^T[col l%16][same k], and holds
// D[rows 4(l/16) .. 4(l/16)+3][col l%16].
//
// Reductions (loss, bias gradients, routing) use a fixed order, so every
// result is reproducible run to run.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "sur_dev.h"

namespace mi355sur {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;

// FP32 -> bfloat16, round to nearest, ties to even (inputs are finite).
__device__ __forceinline__ uint32_t f2bf(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}

__device__ __forceinline__ bf16x8 ld_frag(const uint16_t* p) {
  const uint4 q = *(const uint4*)p;
  return __builtin_bit_cast(bf16x8, q);
}

constexpr float kInvSqrt2Pi = 0.39894228040143268f;

// Prefetch distance (K steps) of the weight fragments in k_mlp_infer.
constexpr int MLP_PD = 3;

// The standard normal distribution function Phi(z), and exp(-z^2 / 2), for
// the exact GELU z Phi(z) and its derivative Phi(z) + z phi(z).  Phi comes
// from the erfc approximation of Abramowitz and Stegun, formula 7.1.26
// (absolute error of erf at most 1.5e-7, against a bfloat16 step of 2^-8 in
// the activations it feeds): with x = |z| / sqrt 2 and t = 1 / (1 + p x),
// erfc(x) = t (a1 + t (a2 + t (a3 + t (a4 + t a5)))) exp(-x^2), and
// Phi(z) = erfc(x) / 2 for z < 0, 1 - erfc(x) / 2 otherwise.  No branch, one
// reciprocal and one exponential per value.
__device__ __forceinline__ float norm_cdf(float z, float& gz) {
  constexpr float kP = 0.3275911f * 0.70710678118654752f;  // p / sqrt 2
  constexpr float c1 = 0.5f * 0.254829592f, c2 = 0.5f * -0.284496736f, c3 = 0.5f * 1.421413741f,
                  c4 = 0.5f * -1.453152027f, c5 = 0.5f * 1.061405429f;  // a_i / 2
  const float t = __builtin_amdgcn_rcpf(fmaf(kP, fabsf(z), 1.0f));
  float s = fmaf(t, c5, c4);
  s = fmaf(t, s, c3);
  s = fmaf(t, s, c2);
  s = fmaf(t, s, c1);
  s *= t;
  gz = __builtin_amdgcn_exp2f(z * z * -0.72134752044448170f);  // 2^(-z^2 log2(e) / 2)
  const float h = s * gz;  // erfc(x) / 2
  return z < 0.0f ? h : 1.0f - h;
}

// Epilogue of a wave's FM x FN fragments at (mw, nw): fragment (i, j) is
// skipped unless vm[i] and vn[j].
template <int EPI, int FM, int FN>
__device__ __forceinline__ void gemm_store(const GemmArgs& g, const f32x4 (&c)[FM][FN], int mw, int nw, int lane,
                                           const bool (&vm)[FM], const bool (&vn)[FN]) {
  const int r16 = lane & 15;
  const int rq = (lane >> 4) * 4;
#pragma unroll
  for (int i = 0; i < FM; ++i) {
    if (!vm[i]) continue;
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      if (!vn[j]) continue;
      const int m0 = mw + 16 * i + rq, n = nw + 16 * j + r16;
      uint32_t t16[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + r;
        const float v = c[i][j][r];
        if (EPI == EPI_GELU_TRAIN || EPI == EPI_GELU_INFER) {
          const float z = v + g.bias[n];
          float gz;
          const float ph = norm_cdf(z, gz);
          t16[r] = f2bf(z * ph);
          g.o16[(size_t)m * g.ld16 + n] = (uint16_t)t16[r];
          if (EPI == EPI_GELU_TRAIN) g.o32[(size_t)m * g.ld32 + n] = ph + z * (gz * kInvSqrt2Pi);
        } else if (EPI == EPI_LINEAR) {
          if (m < g.m_valid) g.o32[(size_t)m * g.ld32 + n] = v + g.bias[n];
        } else if (EPI == EPI_BWD) {
          const float dz = v * g.aux[(size_t)m * g.ldaux + n];
          t16[r] = f2bf(dz);
          g.o16[(size_t)m * g.ld16 + n] = (uint16_t)t16[r];
          g.o32[(size_t)m * g.ld32 + n] = dz;
        } else {  // EPI_DW
          if (n < g.n_valid) g.o32[(size_t)m * g.ld32 + n] = v;
        }
      }
      if (EPI == EPI_GELU_TRAIN || EPI == EPI_BWD)
        *(uint2*)(g.oT + (size_t)n * g.ldT + m0) = make_uint2(t16[0] | (t16[1] << 16), t16[2] | (t16[3] << 16));
    }
  }
}

// One (32 F) x (32 F) output tile per block of four waves; each wave owns a
// (16 F) x (16 F) quarter, F x F fragments.  F = 2 for small products (the
// training batches: more blocks), F = 4 for large ones (twice the reuse of
// every fragment loaded).  Fragments beyond M or N are skipped (the
// conditions are uniform across the wave).  Each accumulator takes its K
// steps in order, so the result does not depend on F.
template <int EPI, int F>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int mw = blockIdx.y * (32 * F) + (w >> 1) * (16 * F);
  const int nw = blockIdx.x * (32 * F) + (w & 1) * (16 * F);
  if (mw >= g.M || nw >= g.N) return;
  bool vm[F], vn[F];
#pragma unroll
  for (int i = 0; i < F; ++i) {
    vm[i] = i == 0 || mw + 16 * i < g.M;
    vn[i] = i == 0 || nw + 16 * i < g.N;
  }
  const int r16 = lane & 15, kq = (lane >> 4) * 8;
  const uint16_t* pa = g.A + (size_t)(mw + r16) * g.lda + kq;
  const uint16_t* pb = g.B + (size_t)(nw + r16) * g.ldb + kq;
  const size_t sa = (size_t)16 * g.lda, sb = (size_t)16 * g.ldb;
  f32x4 c[F][F];
#pragma unroll
  for (int i = 0; i < F; ++i)
#pragma unroll
    for (int j = 0; j < F; ++j) c[i][j] = f32x4{0, 0, 0, 0};
  const bf16x8 zero = __builtin_bit_cast(bf16x8, make_uint4(0, 0, 0, 0));
  // U K steps at a time: all their fragment loads first, then the products,
  // so a wave waits for memory once per U steps.
  auto steps = [&](int k0, auto u_tag) {
    constexpr int U = decltype(u_tag)::value;
    bf16x8 fa[U][F], fb[U][F];
#pragma unroll
    for (int s = 0; s < U; ++s)
#pragma unroll
      for (int i = 0; i < F; ++i) {
        fa[s][i] = vm[i] ? ld_frag(pa + i * sa + k0 + 32 * s) : zero;
        fb[s][i] = vn[i] ? ld_frag(pb + i * sb + k0 + 32 * s) : zero;
      }
#pragma unroll
    for (int s = 0; s < U; ++s)
#pragma unroll
      for (int i = 0; i < F; ++i)
#pragma unroll
        for (int j = 0; j < F; ++j)
          c[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[s][i], fb[s][j], c[i][j], 0, 0, 0);
  };
  constexpr int KU = F == 2 ? 4 : 2;
  int k0 = 0;
  for (; k0 + 32 * KU <= g.K; k0 += 32 * KU) steps(k0, std::integral_constant<int, KU>());
  for (; k0 < g.K; k0 += 32) steps(k0, std::integral_constant<int, 1>());
  gemm_store<EPI, F, F>(g, c, mw, nw, lane, vm, vn);
}

// Large aligned inference products (M and N multiples of 128, K of 64; the
// hidden layers' GELU and the output layer's linear epilogue): the 128 x 128
// output tile of k_gemm<EPI, 4>, four waves of 4 x 4 fragments each, with
// the operands staged through LDS.  K advances in tiles of 64: the block
// copies the 128 x 64 tiles of A and B into LDS once and every wave reads
// its fragments there (in k_gemm two waves fetch each fragment from L2),
// while the loads of the next K tile are in flight in registers.  Rows are
// padded by 16 bytes (144-byte pitch), so the 16 rows of a fragment start
// in 16 distinct groups of four banks.  Each accumulator takes its K steps
// in the same order with the same instruction as k_gemm, and the epilogue
// is k_gemm's: the outputs are the same bits.
constexpr int GL_BM = 128, GL_BK = 64, GL_LD = GL_BK + 8;

// k_gemm_lds's GELU epilogue: gemm_store<EPI_GELU_INFER, 4>'s arithmetic,
// with the bfloat16 outputs staged in the wave's own 64 x 64 slice of LDS
// (lt, pitch GL_LD) so that they leave in 16-byte row pieces instead of one
// 2-byte store per value.
__device__ __forceinline__ void gemm_store_gelu_lds(const GemmArgs& g, const f32x4 (&c)[4][4], int mw, int nw,
                                                    int lane, uint16_t* lt) {
  const int r16 = lane & 15, rq = (lane >> 4) * 4;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int n = nw + 16 * j + r16;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float z = c[i][j][r] + g.bias[n];
        float gz;
        const float ph = norm_cdf(z, gz);
        lt[(16 * i + rq + r) * GL_LD + 16 * j + r16] = (uint16_t)f2bf(z * ph);
      }
    }
  }
  // the slice is this wave's alone: its LDS writes done, its lanes read rows
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  const int ch = (lane & 7) * 8;
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const int row = (lane >> 3) + 8 * t;
    *(uint4*)(g.o16 + (size_t)(mw + row) * g.ld16 + nw + ch) = *(const uint4*)(lt + row * GL_LD + ch);
  }
}

template <int EPI>
__global__ __launch_bounds__(256, 3) void k_gemm_lds(GemmArgs g) {
  __shared__ __attribute__((aligned(16))) uint16_t sm[2 * GL_BM * GL_LD];
  uint16_t* const sa = sm;
  uint16_t* const sb = sm + GL_BM * GL_LD;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  // Blocks are dealt to the 8 XCDs round robin.  The column tiles of one row
  // tile go to one XCD, one after another, so that the row tile of A comes
  // from HBM once and from that XCD's L2 for the other column tiles (dealt
  // in plain order, they would land on N / 128 different XCDs, and each
  // would read it from HBM).
  const int nt = g.N / GL_BM, b = blockIdx.x;
  int mi, ni;
  if ((g.M / GL_BM) % 8 == 0) {
    const int q = b >> 3;
    ni = q % nt;
    mi = (b & 7) + 8 * (q / nt);
  } else {
    mi = b / nt;
    ni = b % nt;
  }
  const int m0 = mi * GL_BM, n0 = ni * GL_BM;
  // this thread's 16-byte pieces of a K tile: rows cr + 32 i, k offset ck
  const int cr = tid >> 3, ck = (tid & 7) * 8;
  const uint16_t* ga = g.A + (size_t)(m0 + cr) * g.lda + ck;
  const uint16_t* gb = g.B + (size_t)(n0 + cr) * g.ldb + ck;
  const size_t a32 = (size_t)32 * g.lda, b32 = (size_t)32 * g.ldb;
  uint16_t* const la = sa + cr * GL_LD + ck;
  uint16_t* const lb = sb + cr * GL_LD + ck;
  // (named values, not arrays: an array would be kept in scratch memory
  // across the asm statement below)
  uint4 a0, a1, a2, a3, b0, b1, b2, b3;
#define GL_FETCH(k0)                             \
  a0 = *(const uint4*)(ga + (k0));               \
  a1 = *(const uint4*)(ga + a32 + (k0));         \
  a2 = *(const uint4*)(ga + 2 * a32 + (k0));     \
  a3 = *(const uint4*)(ga + 3 * a32 + (k0));     \
  b0 = *(const uint4*)(gb + (k0));               \
  b1 = *(const uint4*)(gb + b32 + (k0));         \
  b2 = *(const uint4*)(gb + 2 * b32 + (k0));     \
  b3 = *(const uint4*)(gb + 3 * b32 + (k0));
#define GL_STASH()                               \
  *(uint4*)(la) = a0;                            \
  *(uint4*)(la + 32 * GL_LD) = a1;               \
  *(uint4*)(la + 64 * GL_LD) = a2;               \
  *(uint4*)(la + 96 * GL_LD) = a3;               \
  *(uint4*)(lb) = b0;                            \
  *(uint4*)(lb + 32 * GL_LD) = b1;               \
  *(uint4*)(lb + 64 * GL_LD) = b2;               \
  *(uint4*)(lb + 96 * GL_LD) = b3;
  const int r16 = lane & 15, kq = (lane >> 4) * 8;
  const int wm = (w >> 1) * 64, wn = (w & 1) * 64;
  const uint16_t* fa0 = sa + (wm + r16) * GL_LD + kq;
  const uint16_t* fb0 = sb + (wn + r16) * GL_LD + kq;
  f32x4 c[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) c[i][j] = f32x4{0, 0, 0, 0};
  GL_FETCH(0)
  GL_STASH()
  __syncthreads();
  for (int k0 = 0; k0 < g.K; k0 += GL_BK) {
    const bool more = k0 + GL_BK < g.K;
    if (more) {
      GL_FETCH(k0 + GL_BK)
    }
    // keep the next tile's loads here, ahead of the products (the compiler
    // would otherwise move them down to the LDS stores that use them)
    asm volatile("" ::: "memory");
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      bf16x8 fa[4], fb[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        fa[i] = ld_frag(fa0 + 16 * i * GL_LD + 32 * s);
        fb[i] = ld_frag(fb0 + 16 * i * GL_LD + 32 * s);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          c[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[i], fb[j], c[i][j], 0, 0, 0);
    }
    __syncthreads();  // every wave is done with this tile
    if (more) {
      GL_STASH()
      __syncthreads();
    }
  }
#undef GL_FETCH
#undef GL_STASH
  if (EPI == EPI_GELU_INFER) {
    // the last barrier of the loop has freed the tiles: wave w takes rows
    // [64 w, 64 w + 64) of them
    gemm_store_gelu_lds(g, c, m0 + wm, n0 + wn, lane, sm + w * 64 * GL_LD);
  } else {
    const bool all[4] = {true, true, true, true};
    gemm_store<EPI, 4>(g, c, m0 + wm, n0 + wn, lane, all, all);
  }
}

// Fused inference: every layer of one net over BM rows in one block.  The
// block's activations stay in LDS from layer to layer (bfloat16, rows padded
// by 16 bytes so that the 16 rows of a fragment fall in different banks);
// only the gathered inputs, the weights (a few MB per net, L2-resident) and
// the last layer's FP32 outputs touch memory.  (Layer by layer, a 64K-row
// activation block with 512 x 512 weights moves 128 MB through HBM per
// layer; here it moves none.)  NW waves; the waves split the block's rows
// into NW / (32 / CF) groups and the 32 column fragments of a 512-wide layer
// (16 columns each) into 32 / CF groups: wave w owns the row fragments of
// group w / (32 / CF) and the column fragments c, c + 32 / CF, ... (CF of
// them, c = w % (32 / CF)).  Each activation fragment a wave reads from LDS
// serves CF products, each weight fragment it reads from L2 serves RF.  The
// weight fragments run MLP_PD K steps ahead of the products, the bias of the
// layer is loaded before them.  The K loop has no branches: rows past M hold
// zero inputs, a column fragment past the layer's width multiplies fragment
// 0's weights, and neither result is ever stored.  Each accumulator takes its
// K steps in order with the instruction k_gemm uses, and the epilogue is
// k_gemm's, so the outputs equal the layer-by-layer products bit for bit.
// (At most 64 accumulator registers a lane: 4 waves per SIMD, else 2.)
template <int BM, int NW, int CF>
__global__ __launch_bounds__(64 * NW, (BM / 16) * 32 / NW * 4 <= 64 ? 4 : 2) void k_mlp_infer(MlpArgs a) {
  constexpr int NT = 64 * NW, NWC = 32 / CF, NWR = NW / NWC, RF = BM / 16 / NWR;
  static_assert(NWC * CF == 32 && NWR * NWC == NW && RF * NWR * 16 == BM, "block shape");
  __shared__ __attribute__((aligned(16))) uint16_t act[BM * MLP_LDA];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int cg = w % NWC, r0 = (w / NWC) * RF;  // column group, first row fragment
  const int net = blockIdx.y, m0 = blockIdx.x * BM;
  const uint16_t* bfn = a.bf + (size_t)net * a.bf_stride;
  const float* pn = a.p + (size_t)net * a.p_stride;
  for (int e = tid; e < BM * 4; e += NT) {  // inputs: 32 bfloat16 per row, as four 16-byte pieces
    const int r = e >> 2, q = e & 3;
    uint4 v = make_uint4(0, 0, 0, 0);
    if (m0 + r < a.M) v = *(const uint4*)(a.X16 + (size_t)(m0 + r) * 32 + q * 8);
    *(uint4*)(act + r * MLP_LDA + q * 8) = v;
  }
  __syncthreads();
  const int r16 = lane & 15, kq = (lane >> 4) * 8, rq = (lane >> 4) * 4;
  const uint16_t* pa = act + (16 * r0 + r16) * MLP_LDA + kq;
#pragma unroll 1
  for (int l = 0; l < a.L; ++l) {
    const MlpLayer ly = a.lay[l];
    const int nf = ly.n >> 4;
    // a fragment past the width reads fragment 0's rows and bias (its
    // products are never stored)
    bool vn[CF];
    const uint16_t* pb[CF];
    float bn[CF];
#pragma unroll
    for (int j = 0; j < CF; ++j) {
      vn[j] = cg + NWC * j < nf;
      const int f = vn[j] ? cg + NWC * j : 0;
      pb[j] = bfn + ly.w16 + (size_t)(f * 16 + r16) * ly.kp + kq;
      bn[j] = pn[ly.bias + f * 16 + r16];
    }
    f32x4 c[RF][CF];
#pragma unroll
    for (int i = 0; i < RF; ++i)
#pragma unroll
      for (int j = 0; j < CF; ++j) c[i][j] = f32x4{0, 0, 0, 0};
    // One K step: the wave's activation fragments from LDS, RF x CF products
    // with this step's weight fragments.
    auto kstep = [&](int k0, const bf16x8* b) {
      bf16x8 fa[RF];
#pragma unroll
      for (int i = 0; i < RF; ++i) fa[i] = *(const bf16x8*)(pa + 16 * i * MLP_LDA + k0);
#pragma unroll
      for (int i = 0; i < RF; ++i)
#pragma unroll
        for (int j = 0; j < CF; ++j) c[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[i], b[j], c[i][j], 0, 0, 0);
    };
    // The empty asm statements between steps keep each load in the step that
    // issues it: nothing is stored in the loop, so the compiler would
    // otherwise move the loads down to the step that uses them, and every
    // step would wait for its own loads.
    if (ly.kp == MLP_KMAX) {
      // the 16 steps of a 512-wide layer unrolled: step s reads the register
      // set s % MLP_PD, so the prefetched values are never copied (a copy
      // would wait for the load)
      constexpr int NS = MLP_KMAX / 32;
      bf16x8 b[MLP_PD][CF];
#pragma unroll
      for (int q = 0; q < MLP_PD; ++q)
#pragma unroll
        for (int j = 0; j < CF; ++j) b[q][j] = ld_frag(pb[j] + 32 * q);
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        asm volatile("" ::: "memory");
        kstep(32 * s, b[s % MLP_PD]);
        if (s + MLP_PD < NS)
#pragma unroll
          for (int j = 0; j < CF; ++j) b[s % MLP_PD][j] = ld_frag(pb[j] + 32 * (s + MLP_PD));
      }
    } else {
      // other widths (the first layer, small nets): one step at a time
#pragma unroll 1
      for (int k0 = 0; k0 < ly.kp; k0 += 32) {
        asm volatile("" ::: "memory");
        bf16x8 b[CF];
#pragma unroll
        for (int j = 0; j < CF; ++j) b[j] = ld_frag(pb[j] + k0);
        kstep(k0, b);
      }
    }
    __syncthreads();  // every wave has read this layer's input
    if (l + 1 < a.L) {  // hidden layer: bias, exact GELU, bfloat16 into LDS
#pragma unroll
      for (int j = 0; j < CF; ++j) {
        if (!vn[j]) continue;
        const int n = (cg + NWC * j) * 16 + r16;
#pragma unroll
        for (int i = 0; i < RF; ++i) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const float z = c[i][j][r] + bn[j];
            float gz;
            const float ph = norm_cdf(z, gz);
            act[(16 * (r0 + i) + rq + r) * MLP_LDA + n] = (uint16_t)f2bf(z * ph);
          }
        }
      }
    } else {  // output layer: bias, FP32 staged in LDS, then rows < m_valid out as whole rows
      float* of = (float*)act;
#pragma unroll
      for (int j = 0; j < CF; ++j) {
        if (!vn[j]) continue;
        const int n = (cg + NWC * j) * 16 + r16;
#pragma unroll
        for (int i = 0; i < RF; ++i)
#pragma unroll
          for (int r = 0; r < 4; ++r) of[(16 * (r0 + i) + rq + r) * ly.n + n] = c[i][j][r] + bn[j];
      }
      __syncthreads();
      const int rows = min(BM, a.m_valid - m0);
      for (int e = tid; e < rows * ly.n; e += NT) {
        const int m = e / ly.n, n = e - m * ly.n;
        a.out[(size_t)net * a.ld_net + (size_t)(m0 + m) * a.ldo + n] = of[e];
      }
    }
    __syncthreads();  // the next layer reads what this one wrote
  }
}

// Batch assembly: inputs to bfloat16, zero-padded to 32 columns and to M rows
// (row-major and transposed), targets to a dense FP32 block.
__global__ void k_gather(const float* __restrict__ x, const float* __restrict__ t, const int* __restrict__ rows,
                         int m_valid, int M, int kin, int W, uint16_t* X16, uint16_t* XT, float* T) {
  const int stride = gridDim.x * blockDim.x;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < M * 32; e += stride) {
    const int m = e >> 5, c = e & 31;
    float v = 0.0f;
    if (m < m_valid && c < kin) {
      const long long r = rows ? rows[m] : m;
      v = x[r * kin + c];
    }
    const uint16_t b = (uint16_t)f2bf(v);
    X16[e] = b;
    if (XT) XT[(size_t)c * M + m] = b;
  }
  if (!T) return;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < M * W; e += stride) {
    const int m = e / W, c = e - m * W;
    float v = 0.0f;
    if (m < m_valid) {
      const long long r = rows ? rows[m] : m;
      v = t[r * W + c];
    }
    T[e] = v;
  }
}

// Mean squared error and its gradient dY = 2 (y - t) / (m_valid W), written
// as FP32, bfloat16 and transposed bfloat16.  Each block covers 64 columns x
// 16 rows and leaves the sum of its squared errors in part[].
__global__ __launch_bounds__(256) void k_loss(const float* __restrict__ y, const float* __restrict__ t, int M,
                                              int m_valid, int W, float scale, uint16_t* g16, uint16_t* gT,
                                              float* dz, float* part) {
  __shared__ float red[256];
  const int n = blockIdx.x * 64 + (threadIdx.x & 63);
  const int m0 = blockIdx.y * 16 + (threadIdx.x >> 6) * 4;
  float s = 0.0f;
  uint32_t q[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int m = m0 + r;
    const size_t e = (size_t)m * W + n;
    const float d = m < m_valid ? y[e] - t[e] : 0.0f;
    s += d * d;
    const float gv = scale * d;
    dz[e] = gv;
    q[r] = f2bf(gv);
    g16[e] = (uint16_t)q[r];
  }
  *(uint2*)(gT + (size_t)n * M + m0) = make_uint2(q[0] | (q[1] << 16), q[2] | (q[3] << 16));
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.y * gridDim.x + blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_loss_final(const float* part, int n, float inv, float* loss) {
  __shared__ float red[256];
  float s = 0.0f;
  for (int i = threadIdx.x; i < n; i += 256) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = red[0] * inv;
}

// Column sums of an M x N FP32 block (bias gradients): 64 columns x 4 row
// slices per block, slices added in a fixed order.
__global__ __launch_bounds__(256) void k_colsum(const float* __restrict__ dz, int M, int N, float* out) {
  __shared__ float red[4][64];
  const int c = threadIdx.x & 63, s = threadIdx.x >> 6;
  const int n = blockIdx.x * 64 + c;
  const int rows = (M + 3) / 4, r0 = s * rows, r1 = min(M, r0 + rows);
  float acc = 0.0f;
  if (n < N)
    for (int m = r0; m < r1; ++m) acc += dz[(size_t)m * N + n];
  red[s][c] = acc;
  __syncthreads();
  if (s == 0 && n < N) out[n] = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
}

// Adam on the flat FP32 parameters of one net (update != 0), then refresh of
// the bfloat16 copies W [n x kp] and W^T [kp x n] used by the products.
__global__ __launch_bounds__(256) void k_adam(AdamArgs a) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= a.P) return;
  float p = a.p[e];
  if (a.update) {
    const float g = a.g[e];
    const float m = a.b1 * a.m[e] + (1.0f - a.b1) * g;
    const float v = a.b2 * a.v[e] + (1.0f - a.b2) * (g * g);
    a.m[e] = m;
    a.v[e] = v;
    p = p - a.lr * (m / a.c1) / (sqrtf(v / a.c2) + a.eps);
    a.p[e] = p;
  }
  int l = 0;
  while (l + 1 < a.nl && e >= a.L[l + 1].off) ++l;
  const AdamLayer& L = a.L[l];
  const int i = e - L.off;
  if (i < L.n * L.k) {
    const int row = i / L.k, col = i - row * L.k;
    const uint16_t b = (uint16_t)f2bf(p);
    a.bf[L.w16 + (long long)row * L.kp + col] = b;
    a.bf[L.wt + (long long)col * L.n + row] = b;
  }
}

// Ensemble reduction of one chunk: one wave per row, one pass over the nets'
// outputs ys ([net][row][col], net stride ld_net).  Each lane keeps the
// running sum of its columns (nets added in order) and the running peak of
// the net in hand; the spread is (max - min) / |mean| of the nets' peaks, the
// peaks summed in net order.  Rows with an input outside [-xbound, xbound]
// get an infinite spread.
__global__ __launch_bounds__(256) void k_route(const float* __restrict__ ys, int nets, long long ld_net, int m, int W,
                                               const float* __restrict__ x, int kin, float xbound, float* ymean,
                                               float* spread) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= m) return;
  // an input outside [-xbound, xbound] routes the row whatever the spread
  const bool out = lane < kin && !(fabsf(x[(long long)row * kin + lane]) <= xbound);
  const bool any_out = __ballot(out) != 0;
  constexpr int CMAX = 8;  // columns per lane per group of 512 held in registers
  float pkq[16];           // per net (nets <= 16): the lane's running peak
#pragma unroll
  for (int q = 0; q < 16; ++q) pkq[q] = -INFINITY;
  for (int c0 = 0; c0 < W; c0 += 64 * CMAX) {
    float s[CMAX];
#pragma unroll
    for (int t = 0; t < CMAX; ++t) s[t] = 0.0f;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      if (q < nets) {
        const float* yq = ys + q * ld_net + (long long)row * W;
#pragma unroll
        for (int t = 0; t < CMAX; ++t) {
          const int c = c0 + lane + 64 * t;
          if (c < W) {
            const float v = yq[c];
            s[t] += v;
            pkq[q] = fmaxf(pkq[q], v);
          }
        }
      }
    }
#pragma unroll
    for (int t = 0; t < CMAX; ++t) {
      const int c = c0 + lane + 64 * t;
      if (c < W) ymean[(long long)row * W + c] = s[t] / (float)nets;
    }
  }
  float pmax = -INFINITY, pmin = INFINITY, psum = 0.0f;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    if (q < nets) {
      float pk = pkq[q];
      for (int o = 32; o > 0; o >>= 1) pk = fmaxf(pk, __shfl_xor(pk, o, 64));
      pmax = fmaxf(pmax, pk);
      pmin = fminf(pmin, pk);
      psum += pk;
    }
  }
  if (lane == 0) spread[row] = any_out ? INFINITY : (pmax - pmin) / fabsf(psum / (float)nets);
}

// k_route for four nets and W a multiple of 4: a lane takes 4 adjacent
// columns, with 16-byte loads and no branch around them.  Each column's sum
// runs over the nets in the same order from 0, the peaks are exact maxima,
// and the spread is formed as in k_route: the same bits.
__global__ __launch_bounds__(256) void k_route4(const float* __restrict__ ys, long long ld_net, int m, int W,
                                                const float* __restrict__ x, int kin, float xbound, float* ymean,
                                                float* spread) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= m) return;
  const bool out = lane < kin && !(fabsf(x[(long long)row * kin + lane]) <= xbound);
  const bool any_out = __ballot(out) != 0;
  float pk0 = -INFINITY, pk1 = -INFINITY, pk2 = -INFINITY, pk3 = -INFINITY;
  const float* y0 = ys + (long long)row * W;
  for (int c = 4 * lane; c < W; c += 256) {
    const float4 v0 = *(const float4*)(y0 + c);
    const float4 v1 = *(const float4*)(y0 + ld_net + c);
    const float4 v2 = *(const float4*)(y0 + 2 * ld_net + c);
    const float4 v3 = *(const float4*)(y0 + 3 * ld_net + c);
    float4 sm;
    sm.x = (((0.0f + v0.x) + v1.x) + v2.x) + v3.x;
    sm.y = (((0.0f + v0.y) + v1.y) + v2.y) + v3.y;
    sm.z = (((0.0f + v0.z) + v1.z) + v2.z) + v3.z;
    sm.w = (((0.0f + v0.w) + v1.w) + v2.w) + v3.w;
    *(float4*)(ymean + (long long)row * W + c) =
        make_float4(sm.x / 4.0f, sm.y / 4.0f, sm.z / 4.0f, sm.w / 4.0f);
    pk0 = fmaxf(pk0, fmaxf(fmaxf(v0.x, v0.y), fmaxf(v0.z, v0.w)));
    pk1 = fmaxf(pk1, fmaxf(fmaxf(v1.x, v1.y), fmaxf(v1.z, v1.w)));
    pk2 = fmaxf(pk2, fmaxf(fmaxf(v2.x, v2.y), fmaxf(v2.z, v2.w)));
    pk3 = fmaxf(pk3, fmaxf(fmaxf(v3.x, v3.y), fmaxf(v3.z, v3.w)));
  }
  for (int o = 32; o > 0; o >>= 1) {
    pk0 = fmaxf(pk0, __shfl_xor(pk0, o, 64));
    pk1 = fmaxf(pk1, __shfl_xor(pk1, o, 64));
    pk2 = fmaxf(pk2, __shfl_xor(pk2, o, 64));
    pk3 = fmaxf(pk3, __shfl_xor(pk3, o, 64));
  }
  float pmax = -INFINITY, pmin = INFINITY, psum = 0.0f;
  pmax = fmaxf(pmax, pk0), pmin = fminf(pmin, pk0), psum += pk0;
  pmax = fmaxf(pmax, pk1), pmin = fminf(pmin, pk1), psum += pk1;
  pmax = fmaxf(pmax, pk2), pmin = fminf(pmin, pk2), psum += pk2;
  pmax = fmaxf(pmax, pk3), pmin = fminf(pmin, pk3), psum += pk3;
  if (lane == 0) spread[row] = any_out ? INFINITY : (pmax - pmin) / fabsf(psum / 4.0f);
}

// Ordered list of the rows whose spread is above the threshold or not
// finite, in one block of 1024 threads.  Thread t owns the contiguous rows
// [t L, t L + L), L a multiple of 64 (64 for up to 65,536 rows).  It flags
// them 64 at a time into a bit mask (16 16-byte loads issued together), and
// a block scan of the counts gives each thread's first position.  The thread
// then writes its rows in order from the masks (the first segment's mask is
// kept, later ones are read again).
__device__ __forceinline__ unsigned long long flag_mask(const float* __restrict__ spread, int s, int b, float thr) {
  unsigned long long m = 0;
  if (s + 64 <= b) {
    float4 v[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) v[j] = *(const float4*)(spread + s + 4 * j);
#pragma unroll
    for (int j = 0; j < 16; ++j)
      m |= ((unsigned long long)!(v[j].x <= thr) << (4 * j)) | ((unsigned long long)!(v[j].y <= thr) << (4 * j + 1)) |
           ((unsigned long long)!(v[j].z <= thr) << (4 * j + 2)) | ((unsigned long long)!(v[j].w <= thr) << (4 * j + 3));
  } else {
    for (int r = s; r < b; ++r) m |= (unsigned long long)!(spread[r] <= thr) << (r - s);
  }
  return m;
}

__global__ __launch_bounds__(1024) void k_compact_chunks(const float* __restrict__ spread, int n, float thr,
                                                         int* __restrict__ ids, int* __restrict__ count) {
  __shared__ int wsum[16];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int L = (((n + 1023) / 1024) + 63) & ~63;
  const int a = min(t * L, n), b = min(a + L, n);
  const unsigned long long m0 = a < b ? flag_mask(spread, a, b, thr) : 0ull;
  int c = __popcll(m0);
  for (int s = a + 64; s < b; s += 64) c += __popcll(flag_mask(spread, s, b, thr));
  int incl = c;  // inclusive scan within the wave
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y;
  }
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  int base = 0;
  for (int q = 0; q < w; ++q) base += wsum[q];
  if (t == 1023) *count = base + incl;
  int pos = base + incl - c;
  for (int s = a; s < b; s += 64) {
    unsigned long long m = s == a ? m0 : flag_mask(spread, s, b, thr);
    while (m) {
      ids[pos++] = s + __builtin_ctzll(m);
      m &= m - 1;
    }
  }
}

// Ordered list of the rows whose spread is above the threshold or not finite,
// in one block of 16 waves: the spreads are read 64 at a time (one per lane,
// coalesced), counted by ballot, the counts of the 64-row pieces scanned in
// LDS, and the rows written at their piece's offset plus their rank in it.
__global__ __launch_bounds__(1024) void k_compact(const float* __restrict__ spread, int n, float thr, int* ids,
                                                  int* count) {
  __shared__ int cnt[1024];
  __shared__ int off[1024];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int pieces = (n + 63) / 64;
  const int per = (pieces + 1023) / 1024;   // pieces per scan slot
  for (int s = threadIdx.x; s < 1024; s += 1024) cnt[s] = 0;
  __syncthreads();
  for (int p = w; p < pieces; p += 16) {
    const int i = p * 64 + lane;
    const bool f = i < n && !(spread[i] <= thr);
    const int c = __popcll(__ballot(f));
    if (lane == 0) atomicAdd(&cnt[p / per], c);
  }
  __syncthreads();
  const int mine = cnt[threadIdx.x];
  int v = mine;
  for (int o = 1; o < 1024; o <<= 1) {  // inclusive Hillis-Steele scan
    __syncthreads();
    off[threadIdx.x] = v;
    __syncthreads();
    if (threadIdx.x >= o) v += off[threadIdx.x - o];
  }
  __syncthreads();
  off[threadIdx.x] = v - mine;  // exclusive offset of scan slot
  __syncthreads();
  if (threadIdx.x == 1023) *count = v;
  // each scan slot's pieces in order, by one wave
  for (int slot = w; slot < 1024; slot += 16) {
    int pos = off[slot];
    for (int p = slot * per; p < min(pieces, (slot + 1) * per); ++p) {
      const int i = p * 64 + lane;
      const bool f = i < n && !(spread[i] <= thr);
      const unsigned long long b = __ballot(f);
      if (f) ids[pos + __popcll(b & ((1ull << lane) - 1ull))] = i;
      pos += __popcll(b);
    }
  }
}

static int last() { return (int)hipGetLastError(); }

template <int F>
void launch_gemm_f(int epi, const GemmArgs& a, hipStream_t s) {
  const dim3 grid((a.N + 32 * F - 1) / (32 * F), (a.M + 32 * F - 1) / (32 * F)), block(256);
  switch (epi) {
    case EPI_GELU_TRAIN: k_gemm<EPI_GELU_TRAIN, F><<<grid, block, 0, s>>>(a); break;
    case EPI_GELU_INFER: k_gemm<EPI_GELU_INFER, F><<<grid, block, 0, s>>>(a); break;
    case EPI_LINEAR: k_gemm<EPI_LINEAR, F><<<grid, block, 0, s>>>(a); break;
    case EPI_BWD: k_gemm<EPI_BWD, F><<<grid, block, 0, s>>>(a); break;
    default: k_gemm<EPI_DW, F><<<grid, block, 0, s>>>(a); break;
  }
}

int launch_gemm(int epi, const GemmArgs& a, void* stream) {
  const hipStream_t s = (hipStream_t)stream;
  // 128 x 128 block tiles once they still give every CU a few blocks; the
  // inference products staged through LDS where the shape is aligned to the
  // tiles
  if ((long long)((a.M + 127) / 128) * ((a.N + 127) / 128) >= 1024) {
    const bool infer = epi == EPI_GELU_INFER || epi == EPI_LINEAR;
    if (infer && a.M % GL_BM == 0 && a.N % GL_BM == 0 && a.K % GL_BK == 0 && a.K > 0 &&
        (epi == EPI_LINEAR || a.ld16 % 8 == 0)) {
      const dim3 grid((a.N / GL_BM) * (a.M / GL_BM)), block(256);
      if (epi == EPI_GELU_INFER)
        k_gemm_lds<EPI_GELU_INFER><<<grid, block, 0, s>>>(a);
      else
        k_gemm_lds<EPI_LINEAR><<<grid, block, 0, s>>>(a);
    } else {
      launch_gemm_f<4>(epi, a, s);
    }
  } else {
    launch_gemm_f<2>(epi, a, s);
  }
  return last();
}

int launch_mlp_infer(const MlpArgs& a, int nets, void* stream) {
  if (a.M <= 0) return 0;
  k_mlp_infer<MLP_BM, MLP_NW, MLP_CF><<<dim3((a.M + MLP_BM - 1) / MLP_BM, nets), 64 * MLP_NW, 0, (hipStream_t)stream>>>(a);
  return last();
}

int launch_gather(const float* x, const float* t, const int* rows, int m_valid, int M, int kin, int W,
                  uint16_t* X16, uint16_t* XT, float* T, void* stream) {
  const long long work = (long long)M * (T ? (W > 32 ? W : 32) : 32);
  const int blocks = (int)((work + 255) / 256 < 4096 ? (work + 255) / 256 : 4096);
  k_gather<<<blocks, 256, 0, (hipStream_t)stream>>>(x, t, rows, m_valid, M, kin, W, X16, XT, T);
  return last();
}

int loss_parts(int M, int W) { return (W / 64) * (M / 16); }

int launch_loss(const float* y, const float* t, int M, int m_valid, int W, uint16_t* g16, uint16_t* gT, float* dz,
                float* part, float* loss_dev, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  const double denom = (double)m_valid * W;
  k_loss<<<dim3(W / 64, M / 16), 256, 0, s>>>(y, t, M, m_valid, W, (float)(2.0 / denom), g16, gT, dz, part);
  if (loss_dev) k_loss_final<<<1, 256, 0, s>>>(part, loss_parts(M, W), (float)(1.0 / denom), loss_dev);
  return last();
}

int launch_colsum(const float* dz, int M, int N, float* out, void* stream) {
  k_colsum<<<(N + 63) / 64, 256, 0, (hipStream_t)stream>>>(dz, M, N, out);
  return last();
}

int launch_adam(const AdamArgs& a, void* stream) {
  k_adam<<<(a.P + 255) / 256, 256, 0, (hipStream_t)stream>>>(a);
  return last();
}

int launch_route(const float* ys, int nets, int ld_net, int m, int W, const float* x, int kin, float xbound,
                 float* ymean, float* spread, void* stream) {
  if (m <= 0) return 0;
  const bool vec = nets == 4 && W % 4 == 0 && ld_net % 4 == 0 && ((uintptr_t)ys & 15) == 0 &&
                   ((uintptr_t)ymean & 15) == 0;
  if (vec)
    k_route4<<<(m + 3) / 4, 256, 0, (hipStream_t)stream>>>(ys, ld_net, m, W, x, kin, xbound, ymean, spread);
  else
    k_route<<<(m + 3) / 4, 256, 0, (hipStream_t)stream>>>(ys, nets, ld_net, m, W, x, kin, xbound, ymean, spread);
  return last();
}

int launch_compact(const float* spread, int n, float threshold, int* ids, int* count, void* stream) {
  if (((uintptr_t)spread & 15) == 0)
    k_compact_chunks<<<1, 1024, 0, (hipStream_t)stream>>>(spread, n, threshold, ids, count);
  else
    k_compact<<<1, 1024, 0, (hipStream_t)stream>>>(spread, n, threshold, ids, count);
  return last();
}

}  // namespace mi355sur
