// Host side of the learned pressure guess: buffers, the forward pass, the
// backward pass and Adam on the GPU, and the C ABI entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/cdi.h"
#include "net_internal.h"
#include "net_kernels.h"

using namespace cdinet;

namespace {

struct LayerDesc {
  const char* name;
  int ci, co;   // ci: input channels as stored (padded to 32 for the first layer)
  int ci_used;  // input channels of the master weights
  int level;    // resolution level (0 full, 1 half, ...)
};

constexpr int kLayers = 7;
constexpr LayerDesc kNet[kLayers] = {
    {"e0", 32, 32, 3, 0},    {"e1", 32, 64, 32, 1},   {"e2", 64, 128, 64, 2},
    {"e3", 128, 256, 128, 3}, {"d2", 384, 128, 384, 2}, {"d1", 192, 64, 192, 1},
    {"d0", 96, 32, 96, 0}};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

struct cdi_net {
  int B, H, W;
  hipStream_t stream;
  float* params;   // caller, FP32 master
  float* grads;    // caller, FP32
  // packed weights
  __bf16* wp[kLayers];
  __bf16* wt[kLayers];
  size_t woff[kLayers], boff[kLayers], out_w, out_b;
  // activations
  __bf16 *x0, *e[4], *p[3], *c2, *d2, *c1, *d1, *c0, *d0;
  float* y;
  float* feat;     // FP32 input features [B][3][H][W] (inference path)
  // gradients
  __bf16 *dd0, *dc0, *dd1, *dc1, *dd2, *dc2, *de3, *dp2, *de2, *dp1, *de1, *dp0, *de0;
  float* wpart;    // weight-gradient chunk partials
  size_t wpart_floats;
  float* opart;    // output-layer partials
  float* loss;     // device scalar
  float* target;   // optional device target for training
  bool train;
};

namespace cdinet {

size_t param_count() {
  size_t n = 0;
  for (int l = 0; l < kLayers; ++l) n += (size_t)kNet[l].co * kNet[l].ci_used * 9 + kNet[l].co;
  return n + 32 + 1;
}

namespace {

int chunks_for(int B, int H) {
  int per_b = std::max(1, std::min(H, 32 / std::max(B, 1)));
  return B * per_b;
}

size_t carve(cdi_net* n, char* base, bool train) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* p = base ? base + off : nullptr;
    off = align256(off + bytes);
    return p;
  };
  const size_t B = n->B, H = n->H, W = n->W;
  auto act = [&](int ch, int level) {
    return (__bf16*)take(B * ch * (H >> level) * (W >> level) * sizeof(__bf16));
  };
  for (int l = 0; l < kLayers; ++l) {
    n->wp[l] = (__bf16*)take((size_t)kNet[l].co * 9 * kNet[l].ci * sizeof(__bf16));
    n->wt[l] = (__bf16*)take((size_t)kNet[l].co * 9 * kNet[l].ci * sizeof(__bf16));
  }
  n->feat = (float*)take(B * 3 * H * W * sizeof(float));
  n->e[0] = act(32, 0);
  n->p[0] = act(32, 1);
  n->e[1] = act(64, 1);
  n->p[1] = act(64, 2);
  n->e[2] = act(128, 2);
  n->p[2] = act(128, 3);
  n->e[3] = act(256, 3);
  n->d2 = act(128, 2);
  n->d1 = act(64, 1);
  n->y = (float*)take(B * H * W * sizeof(float));
  n->loss = (float*)take(256);
  n->train = train;
  if (train) {
    // the padded input and the decoder's concatenated inputs, read by the
    // weight gradients
    n->x0 = act(32, 0);
    n->d0 = act(32, 0);
    n->c2 = act(384, 2);
    n->c1 = act(192, 1);
    n->c0 = act(96, 0);
    n->dd0 = act(32, 0); n->dc0 = act(96, 0);
    n->dd1 = act(64, 1); n->dc1 = act(192, 1);
    n->dd2 = act(128, 2); n->dc2 = act(384, 2);
    n->de3 = act(256, 3); n->dp2 = act(128, 3);
    n->de2 = act(128, 2); n->dp1 = act(64, 2);
    n->de1 = act(64, 1); n->dp0 = act(32, 1);
    n->de0 = act(32, 0);
    size_t mx = 0;
    for (int l = 0; l < kLayers; ++l) {
      const int Hl = (int)(H >> kNet[l].level);
      mx = std::max(mx, (size_t)chunks_for((int)B, Hl) * kNet[l].co * kNet[l].ci * 9);
    }
    n->wpart_floats = mx;
    n->wpart = (float*)take(mx * sizeof(float));
    n->opart = (float*)take((size_t)1024 * 34 * sizeof(float));
  }
  return off;
}

unsigned grid1d(size_t n) { return (unsigned)std::min<size_t>(4096, (n + 255) / 256); }
unsigned rows_grid(size_t rows) { return (unsigned)std::min<size_t>(65535, std::max<size_t>(1, rows)); }

// 3x3 convolution at `level`; with xlo the input is cat(up2(xlo), x) read
// in place (clo channels from xlo).
void conv(cdi_net* n, const __bf16* x, const __bf16* w, const float* bias, __bf16* yb, float* yf,
          int ci, int co, int level, int relu, const __bf16* xlo = nullptr, int clo = 0,
          const float* xf = nullptr, const float* ow = nullptr, const float* ob = nullptr,
          float* yo = nullptr) {
  const int H = n->H >> level, W = n->W >> level;
  const int nxt = (W + TPX - 1) / TPX;
  if (co <= 32) {   // 32-channel x 8-row tile: one wave per 2 rows, all 32 channels
    const int rows = CROWS * 4;
    dim3 grid((unsigned)(n->B * ((H + rows - 1) / rows) * nxt), (unsigned)((co + 31) / 32));
    k_conv3_fwd<2, 1><<<grid, NT, 0, n->stream>>>(x, w, bias, yb, yf, n->B, ci, co, H, W, relu, xlo, clo, xf,
                                                   ow, ob, yo);
  } else {          // 64-channel x 4-row tile: 2 waves along the channels, 2 along the rows
    // (the fused output layer is only used on the 32-channel last layer)
    const int rows = CROWS * 2;
    dim3 grid((unsigned)(n->B * ((H + rows - 1) / rows) * nxt), (unsigned)((co + 63) / 64));
    k_conv3_fwd<2, 2><<<grid, NT, 0, n->stream>>>(x, w, bias, yb, yf, n->B, ci, co, H, W, relu, xlo, clo, xf);
  }
}

void pack_weights(cdi_net* n) {
  for (int l = 0; l < kLayers; ++l) {
    const LayerDesc& L = kNet[l];
    const size_t cnt = (size_t)L.co * 9 * L.ci;
    k_pack_w<<<grid1d(cnt), 256, 0, n->stream>>>(n->params + n->woff[l], L.co, L.ci_used, L.ci, n->wp[l], 0);
    if (l > 0)   // the first layer's input gradient is never needed
      k_pack_w<<<grid1d(cnt), 256, 0, n->stream>>>(n->params + n->woff[l], L.co, L.ci_used, L.ci, n->wt[l], 1);
  }
}

}  // namespace

void forward(cdi_net* n) {
  const int B = n->B, H = n->H, W = n->W;
  const size_t HW = (size_t)H * W;
  float* P = n->params;
  // the first layer reads the FP32 features; training also stores the
  // padded BF16 input, which its weight gradient reads
  if (n->train)
    k_pack_input<<<grid1d((size_t)B * 32 * HW), 256, 0, n->stream>>>(n->feat, n->x0, B, (int)HW, 32);
  conv(n, nullptr, n->wp[0], P + n->boff[0], n->e[0], nullptr, 32, 32, 0, 1, nullptr, 0, n->feat);
  k_pool<<<grid1d((size_t)B * 32 * HW / 4), 256, 0, n->stream>>>(n->e[0], n->p[0], B * 32, H, W);
  conv(n, n->p[0], n->wp[1], P + n->boff[1], n->e[1], nullptr, 32, 64, 1, 1);
  k_pool<<<grid1d((size_t)B * 64 * HW / 16), 256, 0, n->stream>>>(n->e[1], n->p[1], B * 64, H / 2, W / 2);
  conv(n, n->p[1], n->wp[2], P + n->boff[2], n->e[2], nullptr, 64, 128, 2, 1);
  k_pool<<<grid1d((size_t)B * 128 * HW / 64), 256, 0, n->stream>>>(n->e[2], n->p[2], B * 128, H / 4, W / 4);
  conv(n, n->p[2], n->wp[3], P + n->boff[3], n->e[3], nullptr, 128, 256, 3, 1);
  // decoder: the convolutions read cat(up2(lo), skip) in place; training
  // also stores the concatenation, which the weight gradient reads
  if (n->train)
    k_upcat<<<rows_grid((size_t)B * 384 * (H / 4)), 256, 0, n->stream>>>(n->e[3], n->e[2], n->c2, B, 256, 128, H / 4, W / 4);
  conv(n, n->e[2], n->wp[4], P + n->boff[4], n->d2, nullptr, 384, 128, 2, 1, n->e[3], 256);
  if (n->train)
    k_upcat<<<rows_grid((size_t)B * 192 * (H / 2)), 256, 0, n->stream>>>(n->d2, n->e[1], n->c1, B, 128, 64, H / 2, W / 2);
  conv(n, n->e[1], n->wp[5], P + n->boff[5], n->d1, nullptr, 192, 64, 1, 1, n->d2, 128);
  if (n->train)
    k_upcat<<<rows_grid((size_t)B * 96 * H), 256, 0, n->stream>>>(n->d1, n->e[0], n->c0, B, 64, 32, H, W);
  // last 3x3 layer (32 channels: one tile holds them all) with the 1x1
  // output layer fused into its epilogue; its activation is stored only for
  // training (the backward pass reads it)
  static_assert(kNet[6].co == 32, "the fused output layer needs a 32-channel last layer");
  conv(n, n->e[0], n->wp[6], P + n->boff[6], n->train ? n->d0 : nullptr, nullptr, 96, 32, 0, 1,
       n->d1, 64, nullptr, P + n->out_w, P + n->out_b, n->y);
}

namespace {

void wgrad(cdi_net* n, int l, const __bf16* x, const __bf16* dy) {
  const LayerDesc& L = kNet[l];
  const int Hl = n->H >> L.level, Wl = n->W >> L.level;
  const int chunks = chunks_for(n->B, Hl);
  const int per_b = chunks / n->B;
  const int rows = (Hl + per_b - 1) / per_b;
  dim3 grid((unsigned)((L.co + TCO - 1) / TCO), (unsigned)(L.ci / KC), (unsigned)chunks);
  k_conv3_wgrad<<<grid, NT, 0, n->stream>>>(x, dy, n->wpart, n->B, L.ci, L.co, Hl, Wl, rows, per_b);
  const size_t cnt = (size_t)L.co * L.ci_used * 9;
  k_wgrad_reduce<<<grid1d(cnt), 256, 0, n->stream>>>(n->wpart, chunks, L.co, L.ci, L.ci_used,
                                                    n->grads + n->woff[l]);
  k_bias_grad<<<(unsigned)L.co, NT, 0, n->stream>>>(dy, n->B, L.co, Hl * Wl, n->grads + n->boff[l]);
}

void relu_bwd(cdi_net* n, __bf16* g, const __bf16* y, int ch, int level) {
  const size_t cnt = (size_t)n->B * ch * (n->H >> level) * (n->W >> level);
  k_relu_bwd<<<grid1d(cnt), 256, 0, n->stream>>>(g, y, cnt);
}

}  // namespace

void backward(cdi_net* n, const float* target) {
  const int B = n->B, H = n->H, W = n->W;
  const size_t HW = (size_t)H * W;
  float* P = n->params;
  float* G = n->grads;
  const unsigned ob = std::min<unsigned>(1024, grid1d((size_t)B * HW));
  k_out_bwd<<<ob, NT, 0, n->stream>>>(n->d0, P + n->out_w, n->y, target, n->dd0, n->opart, B, 32, (int)HW);
  k_out_reduce<<<1, 64, 0, n->stream>>>(n->opart, (int)ob, 32, G + n->out_w, G + n->out_b, n->loss);
  // d0 = relu(conv(c0)): c0 = cat(up(d1), e0)
  relu_bwd(n, n->dd0, n->d0, 32, 0);
  wgrad(n, 6, n->c0, n->dd0);
  conv(n, n->dd0, n->wt[6], nullptr, n->dc0, nullptr, 32, 96, 0, 0);
  k_upcat_bwd_lo<<<grid1d((size_t)B * 64 * HW / 4), 256, 0, n->stream>>>(n->dc0, n->dd1, B, 64, 96, H, W);
  // d1 = relu(conv(c1)): c1 = cat(up(d2), e1)
  relu_bwd(n, n->dd1, n->d1, 64, 1);
  wgrad(n, 5, n->c1, n->dd1);
  conv(n, n->dd1, n->wt[5], nullptr, n->dc1, nullptr, 64, 192, 1, 0);
  k_upcat_bwd_lo<<<grid1d((size_t)B * 128 * HW / 16), 256, 0, n->stream>>>(n->dc1, n->dd2, B, 128, 192, H / 2, W / 2);
  // d2 = relu(conv(c2)): c2 = cat(up(e3), e2)
  relu_bwd(n, n->dd2, n->d2, 128, 2);
  wgrad(n, 4, n->c2, n->dd2);
  conv(n, n->dd2, n->wt[4], nullptr, n->dc2, nullptr, 128, 384, 2, 0);
  k_upcat_bwd_lo<<<grid1d((size_t)B * 256 * HW / 64), 256, 0, n->stream>>>(n->dc2, n->de3, B, 256, 384, H / 4, W / 4);
  // e3 = relu(conv(p2))
  relu_bwd(n, n->de3, n->e[3], 256, 3);
  wgrad(n, 3, n->p[2], n->de3);
  conv(n, n->de3, n->wt[3], nullptr, n->dp2, nullptr, 256, 128, 3, 0);
  // e2 gradient: decoder skip + pooling
  k_skip_grad<<<grid1d((size_t)B * 128 * HW / 16), 256, 0, n->stream>>>(n->dc2, n->dp2, n->de2, B, 256, 128, H / 4, W / 4);
  relu_bwd(n, n->de2, n->e[2], 128, 2);
  wgrad(n, 2, n->p[1], n->de2);
  conv(n, n->de2, n->wt[2], nullptr, n->dp1, nullptr, 128, 64, 2, 0);
  k_skip_grad<<<grid1d((size_t)B * 64 * HW / 4), 256, 0, n->stream>>>(n->dc1, n->dp1, n->de1, B, 128, 64, H / 2, W / 2);
  relu_bwd(n, n->de1, n->e[1], 64, 1);
  wgrad(n, 1, n->p[0], n->de1);
  conv(n, n->de1, n->wt[1], nullptr, n->dp0, nullptr, 64, 32, 1, 0);
  k_skip_grad<<<grid1d((size_t)B * 32 * HW), 256, 0, n->stream>>>(n->dc0, n->dp0, n->de0, B, 64, 32, H, W);
  relu_bwd(n, n->de0, n->e[0], 32, 0);
  wgrad(n, 0, n->x0, n->de0);
}

cdi_status create(const float* params, float* grads, int B, int H, int W, void* ws, size_t bytes,
                  void* stream, bool train, cdi_net** out, std::string& err) {
  *out = nullptr;
  if (!params) { err = "params is NULL"; return CDI_ERR_ARG; }
  if (train && !grads) { err = "grads is NULL"; return CDI_ERR_ARG; }
  if (B < 1 || H < 8 || W < 8 || (H % 8) || (W % 8)) { err = "H, W must be multiples of 8, B >= 1"; return CDI_ERR_SHAPE; }
  if (B > 1024) { err = "batch too large"; return CDI_ERR_ARG; }
  if (!ws || ((uintptr_t)ws & 255)) { err = "workspace NULL or not 256-byte aligned"; return CDI_ERR_ARG; }
  cdi_net tmp{};
  tmp.B = B; tmp.H = H; tmp.W = W;
  const size_t need = carve(&tmp, nullptr, train);
  if (bytes < need) { err = "net workspace too small"; return CDI_ERR_ARG; }
  cdi_net* n = new cdi_net{};
  n->B = B; n->H = H; n->W = W;
  n->stream = (hipStream_t)stream;
  n->params = const_cast<float*>(params);
  n->grads = grads;
  carve(n, (char*)ws, train);
  size_t off = 0;
  for (int l = 0; l < kLayers; ++l) {
    n->woff[l] = off;
    off += (size_t)kNet[l].co * kNet[l].ci_used * 9;
    n->boff[l] = off;
    off += kNet[l].co;
  }
  n->out_w = off;
  n->out_b = off + 32;
  pack_weights(n);
  if (hipGetLastError() != hipSuccess) { delete n; err = "weight packing launch failed"; return CDI_ERR_DEVICE; }
  *out = n;
  return CDI_OK;
}

size_t workspace_bytes(int B, int H, int W, bool train) {
  cdi_net tmp{};
  tmp.B = B; tmp.H = H; tmp.W = W;
  return carve(&tmp, nullptr, train);
}

void pack_weights_public(cdi_net* n) { pack_weights(n); }
float* features(cdi_net* n) { return n->feat; }
float* output(cdi_net* n) { return n->y; }
hipStream_t stream_of(cdi_net* n) { return n->stream; }
int height(cdi_net* n) { return n->H; }
int width(cdi_net* n) { return n->W; }
int batch(cdi_net* n) { return n->B; }

}  // namespace cdinet

// ================================================================ C ABI
namespace {
thread_local std::string g_net_err;
cdi_status net_fail(cdi_status s, const std::string& m) { g_net_err = m; return s; }
}

extern "C" {

size_t cdi_net_param_count(void) { return cdinet::param_count(); }

size_t cdi_net_workspace_bytes(int32_t batch, int32_t h, int32_t w, int32_t train) {
  if (batch < 1 || h < 8 || w < 8 || (h % 8) || (w % 8)) return 0;
  return cdinet::workspace_bytes(batch, h, w, train != 0);
}

cdi_status cdi_net_init(const float* params, float* grads, int32_t batch, int32_t h, int32_t w,
                        int32_t train, void* workspace, size_t workspace_bytes, void* hip_stream,
                        cdi_net** out) {
  if (!out) return net_fail(CDI_ERR_ARG, "out is NULL");
  std::string err;
  cdi_status s = cdinet::create(params, grads, batch, h, w, workspace, workspace_bytes, hip_stream,
                                train != 0, out, err);
  if (s != CDI_OK) g_net_err = err;
  return s;
}

cdi_status cdi_net_repack(cdi_net* n) {
  if (!n) return net_fail(CDI_ERR_ARG, "net is NULL");
  cdinet::pack_weights_public(n);
  return hipGetLastError() == hipSuccess ? CDI_OK : net_fail(CDI_ERR_DEVICE, "launch failed");
}

cdi_status cdi_net_forward(cdi_net* n, const float* x, float* y) {
  if (!n || !x || !y) return net_fail(CDI_ERR_ARG, "NULL argument");
  const size_t HW = (size_t)n->H * n->W;
  if (hipMemcpyAsync(n->feat, x, (size_t)n->B * 3 * HW * sizeof(float), hipMemcpyDeviceToDevice, n->stream) != hipSuccess)
    return net_fail(CDI_ERR_DEVICE, "copy input");
  cdinet::forward(n);
  if (hipMemcpyAsync(y, n->y, (size_t)n->B * HW * sizeof(float), hipMemcpyDeviceToDevice, n->stream) != hipSuccess)
    return net_fail(CDI_ERR_DEVICE, "copy output");
  return hipGetLastError() == hipSuccess ? CDI_OK : net_fail(CDI_ERR_DEVICE, "launch failed");
}

cdi_status cdi_net_backward(cdi_net* n, const float* target, float* loss) {
  if (!n || !target) return net_fail(CDI_ERR_ARG, "NULL argument");
  if (!n->train) return net_fail(CDI_ERR_STATE, "net was created for inference only");
  cdinet::backward(n, target);
  if (loss && hipMemcpyAsync(loss, n->loss, sizeof(float), hipMemcpyDeviceToDevice, n->stream) != hipSuccess)
    return net_fail(CDI_ERR_DEVICE, "copy loss");
  return hipGetLastError() == hipSuccess ? CDI_OK : net_fail(CDI_ERR_DEVICE, "launch failed");
}

cdi_status cdi_net_adam(cdi_net* n, float* m, float* v, int32_t step, double lr) {
  if (!n || !m || !v || step < 1) return net_fail(CDI_ERR_ARG, "bad arguments");
  if (!n->train) return net_fail(CDI_ERR_STATE, "net was created for inference only");
  const size_t cnt = cdinet::param_count();
  const float b1 = 0.9f, b2 = 0.999f;
  // bias corrections 1 - beta^step of the FP32 betas the kernel uses, formed
  // in double: beta2^step lies within ~1e-3 of 1, so in FP32 the difference
  // would keep only ~4 significant digits
  const float c1 = (float)(1.0 - std::pow((double)b1, (double)step));
  const float c2 = (float)(1.0 - std::pow((double)b2, (double)step));
  cdinet::k_adam<<<std::min<unsigned>(2048, (unsigned)((cnt + 255) / 256)), 256, 0, n->stream>>>(
      n->params, n->grads, m, v, cnt, (float)lr, b1, b2, 1e-8f, c1, c2);
  cdinet::pack_weights_public(n);
  return hipGetLastError() == hipSuccess ? CDI_OK : net_fail(CDI_ERR_DEVICE, "launch failed");
}

void cdi_net_destroy(cdi_net* n) { delete n; }

const char* cdi_net_last_error(void) { return g_net_err.c_str(); }

}  // extern "C"
