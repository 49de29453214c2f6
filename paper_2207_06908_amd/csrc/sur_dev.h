// sur_dev.h -- host-side view of the surrogate kernels (launchers only).
#pragma once
#include <stdint.h>

namespace mi355sur {

enum Epi {
  EPI_GELU_TRAIN = 0,  // o16 = bf16(gelu(z)), oT = its transpose, o32 = gelu'(z)
  EPI_GELU_INFER = 1,  // o16 = bf16(gelu(z))
  EPI_LINEAR = 2,      // o32 = z (rows < m_valid)
  EPI_BWD = 3,         // dz = acc * aux; o16 = bf16(dz), oT = its transpose, o32 = dz
  EPI_DW = 4,          // o32 = acc for columns < n_valid
};

// C[M x N] = A[M x K] B[N x K]^T (both operands K-contiguous bfloat16),
// FP32 accumulation on the matrix cores, then the epilogue.  M and N are
// multiples of 16, K a multiple of 32, leading dimensions multiples of 8.
struct GemmArgs {
  const uint16_t* A;
  const uint16_t* B;
  int lda, ldb, M, N, K;
  const float* bias;  // [N], z = acc + bias
  uint16_t* o16;
  int ld16;
  uint16_t* oT;
  int ldT;
  float* o32;
  int ld32;
  const float* aux;
  int ldaux;
  int n_valid;
  int m_valid;
};

struct AdamLayer {
  int off, n, k, kp;  // flat offset of W (bias follows), shape, padded K
  long long w16, wt;  // element offsets of the bfloat16 copies W [n x kp], W^T [kp x n]
};

struct AdamArgs {
  float* p;
  float* m;
  float* v;
  const float* g;
  uint16_t* bf;  // base of the bfloat16 copies of this net
  int P, nl, update;
  float lr, b1, b2, eps, c1, c2;
  AdamLayer L[8];
};

// Fused inference (k_mlp_infer): all layers of `nets` consecutive nets over
// M gathered rows, activations kept on chip; hidden widths <= MLP_KMAX, the
// output width <= MLP_NOUT (its FP32 rows are staged in the same LDS).  Net q's bfloat16 weight copies start at bf + q bf_stride,
// its FP32 parameters at p + q p_stride; its outputs go to
// out[q ld_net + row ldo + col] for rows < m_valid.
// Block shape of k_mlp_infer: MLP_BM rows, MLP_NW waves, MLP_CF column
// fragments per wave.
constexpr int MLP_BM = 128, MLP_NW = 16, MLP_CF = 2;
constexpr int MLP_KMAX = 512, MLP_LDA = MLP_KMAX + 8, MLP_NOUT = MLP_LDA / 2;
struct MlpLayer {
  long long w16;   // element offset of W [n x kp] in a net's bfloat16 copies
  int bias;        // offset of b in a net's FP32 parameters
  int kp, n;
};
struct MlpArgs {
  const uint16_t* X16;  // [M x 32]
  const uint16_t* bf;
  const float* p;
  long long bf_stride, p_stride;
  int M, L, m_valid, ldo;
  float* out;
  long long ld_net;
  MlpLayer lay[8];
};
int launch_mlp_infer(const MlpArgs& a, int nets, void* stream);

int launch_gemm(int epi, const GemmArgs& a, void* stream);
int launch_gather(const float* x, const float* t, const int* rows, int m_valid, int M, int kin, int W,
                  uint16_t* X16, uint16_t* XT, float* T, void* stream);
int launch_loss(const float* y, const float* t, int M, int m_valid, int W, uint16_t* g16, uint16_t* gT,
                float* dz, float* part, float* loss_dev, void* stream);
int launch_colsum(const float* dz, int M, int N, float* out, void* stream);
int launch_adam(const AdamArgs& a, void* stream);
// Mean over nets and peak spread per row; a row with an input outside
// [-xbound, xbound] (x: m rows of kin <= 64 inputs) gets an infinite spread.
int launch_route(const float* ys, int nets, int ld_net, int m, int W, const float* x, int kin, float xbound,
                 float* ymean, float* spread, void* stream);
int launch_compact(const float* spread, int n, float threshold, int* ids, int* count, void* stream);
int loss_parts(int M, int W);

}  // namespace mi355sur
