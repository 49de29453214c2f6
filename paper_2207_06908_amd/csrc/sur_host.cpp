// sur_host.cpp -- host side of the surrogate library (C-ABI of include/sur.h).
//
// Owns the layer geometry, carves the caller's workspace into parameter,
// Adam, activation and gradient buffers, and sequences the kernels of
// sur_kernels.hip: forward (one product per layer with the bias/GELU
// epilogue; inference of every net in one fused launch where the widths
// allow), loss, backward (weight-gradient product, bias column sums and the
// input-gradient product with the GELU-derivative epilogue), Adam.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "sur.h"
#include "sur_dev.h"

using namespace mi355sur;

namespace {

constexpr int kMaxLayers = 7;

struct Layer {
  int k, kp, n;              // fan-in, fan-in padded to the product's K step, fan-out
  long long off_w, off_b;    // flat offsets
  long long w16, wt;         // element offsets of the bfloat16 copies inside a net's copy block
};

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

struct sur_ctx {
  std::vector<int> w;
  int L = 0, nets = 0, R = 0, wmax = 0;
  hipStream_t stream = nullptr;
  std::string err;
  std::vector<Layer> lay;
  long long P = 0, nbf = 0;  // FP32 parameters per net, bfloat16 copy elements per net
  // workspace
  char* ws = nullptr;
  size_t ws_bytes = 0, need = 0;
  size_t o_net = 0, net_stride = 0, o_bf = 0;  // o_bf: offset of the copies inside a net block
  size_t o_X16 = 0, o_XT = 0, o_T = 0, o_y = 0, o_part = 0, o_ys = 0;
  size_t o_a16[kMaxLayers] = {}, o_aT[kMaxLayers] = {}, o_gz[kMaxLayers] = {};
  size_t o_g16[2] = {}, o_gT[2] = {}, o_dz[2] = {};
  std::vector<long long> adam_t;
  std::vector<char> ready;
  float xbound = INFINITY;   // routing bound on the inputs (sur_set_input_bound)
  int fused = 1;             // inference by the fused kernel where the widths allow (sur_set_kernel)

  template <typename T>
  T* at(size_t off) const { return (T*)(ws + off); }
  float* p(int net) const { return at<float>(o_net + net * net_stride); }
  float* m(int net) const { return p(net) + P; }
  float* v(int net) const { return p(net) + 2 * P; }
  float* g(int net) const { return p(net) + 3 * P; }
  uint16_t* bf(int net) const { return at<uint16_t>(o_net + net * net_stride + o_bf); }
};

static int fail(sur_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

static int hip_fail(sur_ctx* c, int e, const char* what) {
  return fail(c, SUR_EDEVICE, std::string(what) + ": " + hipGetErrorString((hipError_t)e));
}

extern "C" {

int sur_create(const int* widths, int n_widths, int n_nets, int max_rows, void* hip_stream, sur_ctx** out) {
  if (!widths || !out || n_widths < 2 || n_widths > kMaxLayers + 1 || n_nets < 1 || n_nets > 16 ||
      max_rows < 64 || max_rows > 65536 || max_rows % 64)
    return SUR_EINVAL;
  if (widths[0] < 1 || widths[0] > 32) return SUR_EINVAL;
  for (int i = 1; i < n_widths; ++i)
    if (widths[i] < 64 || widths[i] > 4096 || widths[i] % 64) return SUR_EINVAL;
  sur_ctx* c = new sur_ctx;
  c->w.assign(widths, widths + n_widths);
  c->L = n_widths - 1;
  c->nets = n_nets;
  c->R = max_rows;
  c->stream = (hipStream_t)hip_stream;
  long long off = 0, bf = 0;
  for (int l = 0; l < c->L; ++l) {
    Layer y;
    y.k = c->w[l];
    y.kp = l == 0 ? 32 : c->w[l];
    y.n = c->w[l + 1];
    y.off_w = off;
    y.off_b = off + (long long)y.n * y.k;
    off = y.off_b + y.n;
    y.w16 = bf;
    y.wt = bf + (long long)y.n * y.kp;
    bf = y.wt + (long long)y.n * y.kp;
    c->lay.push_back(y);
    c->wmax = std::max(c->wmax, y.n);
  }
  c->P = off;
  c->nbf = bf;
  // workspace layout
  const size_t R = c->R, W = c->w.back();
  size_t o = 0;
  auto take = [&](size_t bytes) { const size_t r = o; o += align256(bytes); return r; };
  c->o_bf = align256((size_t)4 * c->P * 4);
  c->net_stride = align256(c->o_bf + (size_t)c->nbf * 2);
  c->o_net = take(c->net_stride * c->nets);
  c->o_X16 = take(R * 32 * 2);
  c->o_XT = take(R * 32 * 2);
  c->o_T = take(R * W * 4);
  for (int l = 0; l + 1 < c->L; ++l) {
    const size_t n = c->lay[l].n;
    c->o_a16[l] = take(R * n * 2);
    c->o_aT[l] = take(R * n * 2);
    c->o_gz[l] = take(R * n * 4);
  }
  c->o_y = take(R * W * 4);
  for (int q = 0; q < 2; ++q) {
    c->o_g16[q] = take(R * c->wmax * 2);
    c->o_gT[q] = take(R * c->wmax * 2);
    c->o_dz[q] = take(R * c->wmax * 4);
  }
  c->o_part = take((size_t)loss_parts(c->R, (int)W) * 4);
  c->o_ys = take((size_t)c->nets * R * W * 4);
  c->need = o;
  c->adam_t.assign(c->nets, 0);
  c->ready.assign(c->nets, 0);
  *out = c;
  return SUR_OK;
}

size_t sur_workspace_bytes(const sur_ctx* c) { return c ? c->need : 0; }

int sur_bind_workspace(sur_ctx* c, void* dev, size_t bytes) {
  if (!c || !dev) return fail(c, SUR_EINVAL, "null workspace");
  if ((uintptr_t)dev % 256) return fail(c, SUR_EINVAL, "workspace must be 256-byte aligned");
  if (bytes < c->need) return fail(c, SUR_ENOMEM, "workspace smaller than sur_workspace_bytes()");
  c->ws = (char*)dev;
  c->ws_bytes = bytes;
  std::fill(c->ready.begin(), c->ready.end(), 0);
  return SUR_OK;
}

long long sur_num_params(const sur_ctx* c) { return c ? c->P : 0; }

static AdamArgs adam_args(const sur_ctx* c, int net, int update, float lr) {
  AdamArgs a{};
  a.p = c->p(net);
  a.m = c->m(net);
  a.v = c->v(net);
  a.g = c->g(net);
  a.bf = c->bf(net);
  a.P = (int)c->P;
  a.nl = c->L;
  a.update = update;
  a.lr = lr;
  a.b1 = 0.9f;
  a.b2 = 0.999f;
  a.eps = 1e-8f;
  const long long t = c->adam_t[net];
  a.c1 = (float)(1.0 - std::pow(0.9, (double)t));
  a.c2 = (float)(1.0 - std::pow(0.999, (double)t));
  for (int l = 0; l < c->L; ++l) {
    const Layer& y = c->lay[l];
    a.L[l] = AdamLayer{(int)y.off_w, y.n, y.k, y.kp, y.w16, y.wt};
  }
  return a;
}

static int check_net(sur_ctx* c, int net, bool need_ready) {
  if (!c) return SUR_EINVAL;
  if (net < 0 || net >= c->nets) return fail(c, SUR_EINVAL, "net index out of range");
  if (!c->ws) return fail(c, SUR_ESTATE, "no workspace bound");
  if (need_ready && !c->ready[net]) return fail(c, SUR_ESTATE, "parameters of this net were never set");
  return SUR_OK;
}

// Upload parameters, clear the Adam state and the bfloat16 copies (their
// padding columns must be zero), then rebuild the copies.
static int upload_params(sur_ctx* c, int net, const float* host) {
  hipError_t e = hipMemcpyAsync(c->p(net), host, (size_t)c->P * 4, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->m(net), 0, (size_t)c->P * 4 * 3, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->bf(net), 0, (size_t)c->nbf * 2, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "parameter upload");
  int r = launch_adam(adam_args(c, net, 0, 0.0f), c->stream);
  if (r) return hip_fail(c, r, "copy refresh");
  e = hipStreamSynchronize(c->stream);  // the host buffer may go away after return
  if (e != hipSuccess) return hip_fail(c, e, "parameter upload");
  c->adam_t[net] = 0;
  c->ready[net] = 1;
  return SUR_OK;
}

static uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

int sur_init_params(sur_ctx* c, int net, unsigned long long seed) {
  int r = check_net(c, net, false);
  if (r) return r;
  std::vector<float> h((size_t)c->P);
  for (const Layer& y : c->lay) {
    const double bound = 1.0 / std::sqrt((double)y.k);
    for (long long i = y.off_w; i < y.off_b + y.n; ++i) {
      const uint64_t z = splitmix64(seed * 0xD1B54A32D192ED03ull + (uint64_t)i);
      const double u = (double)(z >> 11) * 0x1.0p-53;
      h[(size_t)i] = (float)((2.0 * u - 1.0) * bound);
    }
  }
  return upload_params(c, net, h.data());
}

int sur_set_params(sur_ctx* c, int net, const float* host) {
  int r = check_net(c, net, false);
  if (r) return r;
  if (!host) return fail(c, SUR_EINVAL, "null parameters");
  return upload_params(c, net, host);
}

static int download(sur_ctx* c, const float* dev, float* host) {
  if (!host) return fail(c, SUR_EINVAL, "null output");
  hipError_t e = hipMemcpyAsync(host, dev, (size_t)c->P * 4, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "download");
  return SUR_OK;
}

int sur_get_params(sur_ctx* c, int net, float* host) {
  int r = check_net(c, net, true);
  return r ? r : download(c, c->p(net), host);
}

int sur_get_grads(sur_ctx* c, int net, float* host) {
  int r = check_net(c, net, true);
  return r ? r : download(c, c->g(net), host);
}

// Forward pass of rows already gathered into X16 (M rows, multiple of 64).
// train: keep every activation, its transpose and the GELU derivative.
static int forward(sur_ctx* c, int net, int M, bool train, float* y, int ldy, int m_valid) {
  const uint16_t* in = c->at<uint16_t>(c->o_X16);
  const uint16_t* bfb = c->bf(net);
  for (int l = 0; l < c->L; ++l) {
    const Layer& ly = c->lay[l];
    GemmArgs a{};
    a.A = in;
    a.lda = ly.kp;
    a.B = bfb + ly.w16;
    a.ldb = ly.kp;
    a.M = M;
    a.N = ly.n;
    a.K = ly.kp;
    a.bias = c->p(net) + ly.off_b;
    int epi;
    if (l + 1 < c->L) {
      epi = train ? EPI_GELU_TRAIN : EPI_GELU_INFER;
      a.o16 = c->at<uint16_t>(c->o_a16[l]);
      a.ld16 = ly.n;
      a.oT = c->at<uint16_t>(c->o_aT[l]);
      a.ldT = M;
      a.o32 = c->at<float>(c->o_gz[l]);
      a.ld32 = ly.n;
      in = a.o16;
    } else {
      epi = EPI_LINEAR;
      a.o32 = y;
      a.ld32 = ldy;
      a.m_valid = m_valid;
    }
    const int e = launch_gemm(epi, a, c->stream);
    if (e) return hip_fail(c, e, "forward product");
  }
  return SUR_OK;
}

// Whether the fused inference kernel takes this geometry: hidden widths up to
// MLP_KMAX, the output width up to MLP_NOUT.
static bool fused_ok(const sur_ctx* c) {
  if (!c->fused) return false;
  for (int l = 0; l < c->L; ++l) {
    const int n = c->lay[l].n;
    if (l + 1 < c->L ? n > MLP_KMAX : n > MLP_NOUT) return false;
  }
  return c->L <= 8;
}

// All layers of nets [net0, net0 + nets) over the M gathered rows of X16, in
// one launch; outputs to y[q ld_net + row W + col] for rows < m_valid.
static int forward_fused(sur_ctx* c, int net0, int nets, int M, float* y, long long ld_net, int m_valid) {
  MlpArgs a{};
  a.X16 = c->at<uint16_t>(c->o_X16);
  a.bf = c->bf(net0);
  a.p = c->p(net0);
  a.bf_stride = (long long)(c->net_stride / 2);
  a.p_stride = (long long)(c->net_stride / 4);
  a.M = M;
  a.L = c->L;
  a.m_valid = m_valid;
  a.ldo = c->w.back();
  a.out = y;
  a.ld_net = ld_net;
  for (int l = 0; l < c->L; ++l) {
    const Layer& ly = c->lay[l];
    a.lay[l] = MlpLayer{ly.w16, (int)ly.off_b, ly.kp, ly.n};
  }
  const int e = launch_mlp_infer(a, nets, c->stream);
  return e ? hip_fail(c, e, "fused inference") : SUR_OK;
}

int sur_train_step(sur_ctx* c, int net, const float* x_dev, const float* t_dev, const int* rows_dev, int batch,
                   float lr, int update, float* loss_dev) {
  int r = check_net(c, net, true);
  if (r) return r;
  if (!x_dev || !t_dev || batch < 1 || batch > c->R) return fail(c, SUR_EINVAL, "bad batch");
  if (!(lr >= 0.0f) || !std::isfinite(lr)) return fail(c, SUR_EINVAL, "bad learning rate");
  const int M = (batch + 63) / 64 * 64, W = c->w.back();
  int e = launch_gather(x_dev, t_dev, rows_dev, batch, M, c->w[0], W, c->at<uint16_t>(c->o_X16),
                        c->at<uint16_t>(c->o_XT), c->at<float>(c->o_T), c->stream);
  if (e) return hip_fail(c, e, "gather");
  if ((r = forward(c, net, M, true, c->at<float>(c->o_y), W, M))) return r;
  e = launch_loss(c->at<float>(c->o_y), c->at<float>(c->o_T), M, batch, W, c->at<uint16_t>(c->o_g16[0]),
                  c->at<uint16_t>(c->o_gT[0]), c->at<float>(c->o_dz[0]), c->at<float>(c->o_part), loss_dev,
                  c->stream);
  if (e) return hip_fail(c, e, "loss");
  int cur = 0;
  for (int l = c->L - 1; l >= 0; --l) {
    const Layer& ly = c->lay[l];
    GemmArgs a{};  // dW_l = dZ_l^T A_{l-1}
    a.A = c->at<uint16_t>(c->o_gT[cur]);
    a.lda = M;
    a.B = l == 0 ? c->at<uint16_t>(c->o_XT) : c->at<uint16_t>(c->o_aT[l - 1]);
    a.ldb = M;
    a.M = ly.n;
    a.N = ly.kp;
    a.K = M;
    a.o32 = c->g(net) + ly.off_w;
    a.ld32 = ly.k;
    a.n_valid = ly.k;
    if ((e = launch_gemm(EPI_DW, a, c->stream))) return hip_fail(c, e, "weight gradient");
    if ((e = launch_colsum(c->at<float>(c->o_dz[cur]), M, ly.n, c->g(net) + ly.off_b, c->stream)))
      return hip_fail(c, e, "bias gradient");
    if (l == 0) break;
    GemmArgs b{};  // dZ_{l-1} = (dZ_l W_l) * gelu'(Z_{l-1})
    b.A = c->at<uint16_t>(c->o_g16[cur]);
    b.lda = ly.n;
    b.B = c->bf(net) + ly.wt;
    b.ldb = ly.n;
    b.M = M;
    b.N = ly.kp;
    b.K = ly.n;
    b.aux = c->at<float>(c->o_gz[l - 1]);
    b.ldaux = ly.kp;
    b.o16 = c->at<uint16_t>(c->o_g16[1 - cur]);
    b.ld16 = ly.kp;
    b.oT = c->at<uint16_t>(c->o_gT[1 - cur]);
    b.ldT = M;
    b.o32 = c->at<float>(c->o_dz[1 - cur]);
    b.ld32 = ly.kp;
    if ((e = launch_gemm(EPI_BWD, b, c->stream))) return hip_fail(c, e, "input gradient");
    cur ^= 1;
  }
  if (update) {
    c->adam_t[net] += 1;
    if ((e = launch_adam(adam_args(c, net, 1, lr), c->stream))) return hip_fail(c, e, "adam");
  }
  return SUR_OK;
}

int sur_forward(sur_ctx* c, int net, const float* x_dev, int n, float* y_dev) {
  int r = check_net(c, net, true);
  if (r) return r;
  if (n < 0 || (n > 0 && (!x_dev || !y_dev))) return fail(c, SUR_EINVAL, "bad forward arguments");
  const int W = c->w.back(), k0 = c->w[0];
  for (int c0 = 0; c0 < n; c0 += c->R) {
    const int m = std::min(c->R, n - c0), M = (m + 63) / 64 * 64;
    int e = launch_gather(x_dev + (size_t)c0 * k0, nullptr, nullptr, m, M, k0, W, c->at<uint16_t>(c->o_X16),
                          nullptr, nullptr, c->stream);
    if (e) return hip_fail(c, e, "gather");
    r = fused_ok(c) ? forward_fused(c, net, 1, M, y_dev + (size_t)c0 * W, 0, m)
                    : forward(c, net, M, false, y_dev + (size_t)c0 * W, W, m);
    if (r) return r;
  }
  return SUR_OK;
}

int sur_infer_route(sur_ctx* c, const float* x_dev, int n, float threshold, float* y_mean_dev, float* spread_dev,
                    int* fallback_dev, int* n_fallback_dev) {
  if (!c) return SUR_EINVAL;
  if (!c->ws) return fail(c, SUR_ESTATE, "no workspace bound");
  for (int q = 0; q < c->nets; ++q)
    if (!c->ready[q]) return fail(c, SUR_ESTATE, "parameters of a net were never set");
  if (n < 0 || !n_fallback_dev || (n > 0 && (!x_dev || !y_mean_dev || !spread_dev || !fallback_dev)))
    return fail(c, SUR_EINVAL, "bad routing arguments");
  const int W = c->w.back(), k0 = c->w[0];
  float* ys = c->at<float>(c->o_ys);
  int r;
  for (int c0 = 0; c0 < n; c0 += c->R) {
    const int m = std::min(c->R, n - c0), M = (m + 63) / 64 * 64;
    int e = launch_gather(x_dev + (size_t)c0 * k0, nullptr, nullptr, m, M, k0, W, c->at<uint16_t>(c->o_X16),
                          nullptr, nullptr, c->stream);
    if (e) return hip_fail(c, e, "gather");
    if (fused_ok(c)) {
      if ((r = forward_fused(c, 0, c->nets, M, ys, (long long)c->R * W, m))) return r;
    } else {
      for (int q = 0; q < c->nets; ++q)
        if ((r = forward(c, q, M, false, ys + (size_t)q * c->R * W, W, m))) return r;
    }
    if ((e = launch_route(ys, c->nets, c->R * W, m, W, x_dev + (size_t)c0 * k0, k0, c->xbound,
                          y_mean_dev + (size_t)c0 * W, spread_dev + c0, c->stream)))
      return hip_fail(c, e, "route");
  }
  int e = launch_compact(spread_dev, n, threshold, fallback_dev, n_fallback_dev, c->stream);
  if (e) return hip_fail(c, e, "compact");
  return SUR_OK;
}

int sur_set_kernel(sur_ctx* c, int fused) {
  if (!c || (fused != 0 && fused != 1)) return fail(c, SUR_EINVAL, "kernel choice must be 0 or 1");
  c->fused = fused;
  return SUR_OK;
}

int sur_set_input_bound(sur_ctx* c, float bound) {
  if (!c) return SUR_EINVAL;
  if (!(bound > 0.0f)) return fail(c, SUR_EINVAL, "input bound must be positive (INFINITY: off)");
  c->xbound = bound;
  return SUR_OK;
}

const char* sur_last_error(const sur_ctx* c) { return c ? c->err.c_str() : "null handle"; }

void sur_destroy(sur_ctx* c) { delete c; }

}  // extern "C"
