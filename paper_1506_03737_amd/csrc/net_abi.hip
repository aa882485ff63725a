// C ABI of the learned displacement correction (declared in include/lpc.h): the layer table of the 3-level U-Net,
// the workspace plan, and the launch sequences of the forward pass, of backpropagation and of the Adam update.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "../../include/lpc.h"
#include "abi_common.h"
#include "net_kernels.h"

namespace {

using lpc::abi::check;
using lpc::abi::fail;
using lpc::abi::guarded;
namespace net = lpc::net;
using net::bf16;
using net::View;

enum Kind { kConv3 = 0, kDown2 = 1, kUp2 = 2 };

struct LayerDef {
  int kind, cin, cout;
};

// The network of include/lpc.h, in parameter order.
enum { E0A, E0B, DOWN1, E1, DOWN2, B2, UP1, C1, UP0, C0, OUT, kNumLayers };
constexpr LayerDef kLayers[kNumLayers] = {
    {kConv3, net::kInputChannels, 16},  {kConv3, 16, 16}, {kDown2, 16, 32}, {kConv3, 32, 32}, {kDown2, 32, 64}, {kConv3, 64, 64},
    {kUp2, 64, 32},   {kConv3, 64, 32}, {kUp2, 32, 16},   {kConv3, 32, 16}, {kConv3, 16, 3},
};

int taps(int kind) { return kind == kConv3 ? 27 : 8; }
int64_t weight_count(const LayerDef& L) { return static_cast<int64_t>(L.cout) * taps(L.kind) * L.cin; }
int64_t layer_offset(int l) {
  int64_t off = 0;
  for (int i = 0; i < l; ++i) off += weight_count(kLayers[i]) + kLayers[i].cout;
  return off;
}
int64_t param_count() { return layer_offset(kNumLayers); }

int round_to(int x, int m) { return (x + m - 1) / m * m; }

// MFMA layouts of a 3^3 layer: forward [16 nbo][kpad] over cinp input channels; flipped [16 nbi][kpadb] over coutp.
struct ConvShape {
  int cinp, nbo, kpad, coutp, nbi, kpadb;
};
ConvShape conv_shape(const LayerDef& L) {
  ConvShape c;
  c.cinp = round_to(L.cin, 8);
  c.nbo = (L.cout + 15) / 16;
  c.kpad = round_to(27 * c.cinp, 32);
  c.coutp = round_to(L.cout, 8);
  c.nbi = (L.cin + 15) / 16;
  c.kpadb = round_to(27 * c.coutp, 32);
  return c;
}

constexpr size_t kAlign = 256;
size_t round_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Workspace of one D^3 sample: activations, their gradients, converted weights, weight-gradient partial sums.
struct NetWs {
  int D = 0;
  int* flags = nullptr;
  bf16 *x = nullptr, *a0 = nullptr, *cat0 = nullptr, *c0 = nullptr, *a1 = nullptr, *cat1 = nullptr, *c1 = nullptr,
       *a2 = nullptr, *b2 = nullptr;
  bf16 *dout = nullptr, *dc0 = nullptr, *dcat0 = nullptr, *da0 = nullptr, *dc1 = nullptr, *dcat1 = nullptr,
       *da1 = nullptr, *db2 = nullptr, *da2 = nullptr;
  float *out = nullptr, *feat = nullptr, *partial = nullptr;
  double* loss_part = nullptr;
  bf16* wf[kNumLayers] = {};
  bf16* wb[kNumLayers] = {};
  float* wt[kNumLayers] = {};  // 2^3 layers: transposed FP32 weights of the data gradient
  size_t total = 0;
};

int64_t partial_floats(int D) {
  int64_t best = 0;
  int Dl[kNumLayers];  // grid side of each layer's base voxels (see net::wgrad)
  Dl[E0A] = Dl[E0B] = Dl[C0] = Dl[OUT] = D;
  Dl[E1] = Dl[C1] = D / 2;
  Dl[B2] = D / 4;
  Dl[DOWN1] = D;          // down2: base voxels on (D/2)^3
  Dl[DOWN2] = D / 2;
  Dl[UP1] = D / 4;      // up2: base voxels on the coarse grid
  Dl[UP0] = D / 2;
  for (int l = 0; l < kNumLayers; ++l) {
    const LayerDef& L = kLayers[l];
    const int nchunk = net::wgrad_chunks(L.kind, round_to(L.cin, 8), L.cout, Dl[l]);
    const int nslot = (L.kind == kUp2) ? 8 : 1;
    best = std::max<int64_t>(best, static_cast<int64_t>(nchunk) * (weight_count(L) + nslot * L.cout));
  }
  return best;
}

NetWs layout(void* base, int D) {
  NetWs w;
  w.D = D;
  const size_t V = static_cast<size_t>(D) * D * D, V1 = V / 8, V2 = V / 64;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* p = base ? static_cast<char*>(base) + off : nullptr;
    off += round_up(bytes);
    return p;
  };
  auto act = [&](size_t vox, int c) { return reinterpret_cast<bf16*>(take(vox * c * sizeof(bf16))); };
  w.flags = reinterpret_cast<int*>(take(4 * sizeof(int)));
  w.x = act(V, 8);
  w.a0 = act(V, 16);
  w.cat0 = act(V, 32);
  w.c0 = act(V, 16);
  w.a1 = act(V1, 32);
  w.cat1 = act(V1, 64);
  w.c1 = act(V1, 32);
  w.a2 = act(V2, 64);
  w.b2 = act(V2, 64);
  w.dout = act(V, 8);
  w.dc0 = act(V, 16);
  w.dcat0 = act(V, 32);
  w.da0 = act(V, 16);
  w.dc1 = act(V1, 32);
  w.dcat1 = act(V1, 64);
  w.da1 = act(V1, 32);
  w.db2 = act(V2, 64);
  w.da2 = act(V2, 64);
  w.out = reinterpret_cast<float*>(take(V * 3 * sizeof(float)));
  w.feat = reinterpret_cast<float*>(take(V * net::kInputChannels * sizeof(float)));
  w.loss_part = reinterpret_cast<double*>(take(static_cast<size_t>(net::loss_blocks(static_cast<int>(V))) * 8));
  w.partial = reinterpret_cast<float*>(take(static_cast<size_t>(partial_floats(D)) * sizeof(float)));
  for (int l = 0; l < kNumLayers; ++l) {
    if (kLayers[l].kind != kConv3) {
      w.wt[l] = reinterpret_cast<float*>(take(static_cast<size_t>(weight_count(kLayers[l])) * sizeof(float)));
      continue;
    }
    const ConvShape c = conv_shape(kLayers[l]);
    w.wf[l] = reinterpret_cast<bf16*>(take(static_cast<size_t>(16 * c.nbo) * c.kpad * sizeof(bf16)));
    w.wb[l] = reinterpret_cast<bf16*>(take(static_cast<size_t>(16 * c.nbi) * c.kpadb * sizeof(bf16)));
  }
  w.total = off;
  return w;
}

bool size_ok(int D) { return D >= 8 && D <= 512 && (D % 4) == 0; }

// The down/up layers read weights as 16-byte vectors (every layer's W starts at a multiple of 8 values).
lpc_status check_params(const float* params) {
  if (reinterpret_cast<uintptr_t>(params) % 16 != 0) return fail(LPC_ERR_INVALID_ARG, "params must be 16-byte aligned");
  return LPC_OK;
}

lpc_status check_net_ws(int D, void* ws, size_t ws_bytes, NetWs* out) {
  if (!size_ok(D)) return fail(LPC_ERR_UNSUPPORTED_SIZE, "n_side = %d: need a multiple of 4 in [8, 512]", D);
  if (!ws) return fail(LPC_ERR_INVALID_ARG, "workspace pointer is NULL");
  if (reinterpret_cast<uintptr_t>(ws) % kAlign != 0) return fail(LPC_ERR_WORKSPACE, "workspace not 256-byte aligned");
  const NetWs w = layout(ws, D);
  if (ws_bytes < w.total) return fail(LPC_ERR_WORKSPACE, "workspace too small: %zu bytes given, %zu needed", ws_bytes, w.total);
  *out = w;
  return LPC_OK;
}

const float* Wp(const float* params, int l) { return params + layer_offset(l); }
const float* Bp(const float* params, int l) { return params + layer_offset(l) + weight_count(kLayers[l]); }

View v(bf16* p, int ld, int off = 0) { return View{p, ld, off}; }

// BF16 copies of every 3^3 layer's weights (forward and flipped; the first layer's flipped copy is never used).
void convert_weights(const NetWs& w, const float* params, hipStream_t s) {
  for (int l = 0; l < kNumLayers; ++l) {
    const LayerDef& L = kLayers[l];
    if (L.kind != kConv3) {
      check(net::transpose2(Wp(params, l), L.cout, L.cin, w.wt[l], s), "transpose weights");
      continue;
    }
    const ConvShape c = conv_shape(L);
    check(net::convert_conv3(Wp(params, l), L.cout, L.cin, w.wf[l], c.cinp, c.nbo, c.kpad, w.wb[l], c.coutp, c.nbi,
                             c.kpadb, s),
          "convert weights");
  }
}

void conv_fwd(const NetWs& w, const float* params, int l, View in, View out, float* outf, int D, hipStream_t s) {
  const LayerDef& L = kLayers[l];
  const ConvShape c = conv_shape(L);
  check(net::conv3(in, c.cinp, w.wf[l], c.kpad, c.nbo, Bp(params, l), outf ? 0 : 1, out, outf, L.cout, D, s),
        "conv3 forward");
}

// data gradient of 3^3 layer l: dx[.][cin] = conv3(dz[.][coutp], flipped weights)
// (channels below mask_ch then get the leaky-ReLU gradient of the activation view mask)
void conv_dgrad(const NetWs& w, int l, View dz, View dx, int D, hipStream_t s, View mask, int mask_ch) {
  const LayerDef& L = kLayers[l];
  const ConvShape c = conv_shape(L);
  check(net::conv3(dz, c.coutp, w.wb[l], c.kpadb, c.nbi, nullptr, 0, dx, nullptr, L.cin, D, s, mask, mask_ch),
        "conv3 data grad");
}

void weight_grad(const NetWs& w, int l, View x, int cin, View dz, int D, float* grad, hipStream_t s) {
  const LayerDef& L = kLayers[l];
  check(net::wgrad(L.kind, x, cin, L.cin, dz, L.cout, D, w.partial, s), "weight grad");
  const int nchunk = net::wgrad_chunks(L.kind, cin, L.cout, D);
  const int nslot = (L.kind == kUp2) ? 8 : 1;
  check(net::reduce_partials(w.partial, nchunk, static_cast<int>(weight_count(L)), L.cout, nslot, grad + layer_offset(l),
                             s),
        "reduce weight grad");
}

// Forward pass of the feature grid w.feat (FP32 [V][6]) into w.out (FP32 [V][3]); with input_packed the BF16 network
// input w.x is already written (features_packed) and w.feat is not read.
void forward(const NetWs& w, const float* params, hipStream_t s, bool input_packed = false) {
  const int D = w.D, Dh = D / 2, Dq = D / 4;
  const int V = D * D * D;
  convert_weights(w, params, s);
  if (!input_packed) check(net::pack_input(w.feat, w.x, V, s), "pack input");
  conv_fwd(w, params, E0A, v(w.x, 8), v(w.a0, 16), nullptr, D, s);
  conv_fwd(w, params, E0B, v(w.a0, 16), v(w.cat0, 32, 16), nullptr, D, s);                       // s0
  check(net::down2(v(w.cat0, 32, 16), 16, Wp(params, DOWN1), Bp(params, DOWN1), 32, v(w.a1, 32), D, s), "down2");
  conv_fwd(w, params, E1, v(w.a1, 32), v(w.cat1, 64, 32), nullptr, Dh, s);                        // s1
  check(net::down2(v(w.cat1, 64, 32), 32, Wp(params, DOWN2), Bp(params, DOWN2), 64, v(w.a2, 64), Dh, s), "down2");
  conv_fwd(w, params, B2, v(w.a2, 64), v(w.b2, 64), nullptr, Dq, s);
  check(net::up2(v(w.b2, 64), 64, Wp(params, UP1), Bp(params, UP1), 32, v(w.cat1, 64, 0), Dq, s), "up2");  // u1
  conv_fwd(w, params, C1, v(w.cat1, 64), v(w.c1, 32), nullptr, Dh, s);
  check(net::up2(v(w.c1, 32), 32, Wp(params, UP0), Bp(params, UP0), 16, v(w.cat0, 32, 0), Dh, s), "up2");  // u0
  conv_fwd(w, params, C0, v(w.cat0, 32), v(w.c0, 16), nullptr, D, s);
  conv_fwd(w, params, OUT, v(w.c0, 16), View{nullptr, 0, 0}, w.out, D, s);
}

// Backpropagation of the loss against target into grad (FP32 [P]); the loss is summed into w.loss_part.
void backward(const NetWs& w, const float* params, const float* target, float* grad, hipStream_t s) {
  const int D = w.D, Dh = D / 2, Dq = D / 4;
  const int V = D * D * D, Vh = V / 8, Vq = V / 64;
  check(net::loss_grad(w.out, target, w.dout, w.loss_part, V, s), "loss grad");
  // Each data gradient applies the leaky-ReLU gradient of the activation it flows into as it is written.
  // out = conv3(c0)
  weight_grad(w, OUT, v(w.c0, 16), 16, v(w.dout, 8), D, grad, s);
  conv_dgrad(w, OUT, v(w.dout, 8), v(w.dc0, 16), D, s, v(w.c0, 16), 16);  // c0 = leaky(conv3([u0, s0]))
  weight_grad(w, C0, v(w.cat0, 32), 32, v(w.dc0, 16), D, grad, s);
  // u0 = leaky(up2(c1)) takes channels 0..15; s0's gradient is complete only after the down layer's part below
  conv_dgrad(w, C0, v(w.dc0, 16), v(w.dcat0, 32), D, s, v(w.cat0, 32, 0), 16);
  weight_grad(w, UP0, v(w.c1, 32), 32, v(w.dcat0, 32, 0), Dh, grad, s);
  // c1 = leaky(conv3([u1, s1]))
  check(net::up2_dgrad(v(w.dcat0, 32, 0), 16, w.wt[UP0], 32, v(w.dc1, 32), Dh, s, v(w.c1, 32), 32), "up2 grad");
  weight_grad(w, C1, v(w.cat1, 64), 64, v(w.dc1, 32), Dh, grad, s);
  // u1 = leaky(up2(b2)) takes channels 0..31
  conv_dgrad(w, C1, v(w.dc1, 32), v(w.dcat1, 64), Dh, s, v(w.cat1, 64, 0), 32);
  weight_grad(w, UP1, v(w.b2, 64), 64, v(w.dcat1, 64, 0), Dq, grad, s);
  // b2 = leaky(conv3(a2))
  check(net::up2_dgrad(v(w.dcat1, 64, 0), 32, w.wt[UP1], 64, v(w.db2, 64), Dq, s, v(w.b2, 64), 64), "up2 grad");
  weight_grad(w, B2, v(w.a2, 64), 64, v(w.db2, 64), Dq, grad, s);
  // a2 = leaky(down2(s1))
  conv_dgrad(w, B2, v(w.db2, 64), v(w.da2, 64), Dq, s, v(w.a2, 64), 64);
  weight_grad(w, DOWN2, v(w.cat1, 64, 32), 32, v(w.da2, 64), Dh, grad, s);
  // s1 = leaky(conv3(a1)) also feeds c1, so its gradient accumulates before the activation's gradient
  check(net::down2_dgrad(v(w.da2, 64), 64, w.wt[DOWN2], 32, v(w.dcat1, 64, 32), Dh, 1, s, v(w.cat1, 64, 32), 32),
        "down2 grad");
  weight_grad(w, E1, v(w.a1, 32), 32, v(w.dcat1, 64, 32), Dh, grad, s);
  // a1 = leaky(down2(s0))
  conv_dgrad(w, E1, v(w.dcat1, 64, 32), v(w.da1, 32), Dh, s, v(w.a1, 32), 32);
  weight_grad(w, DOWN1, v(w.cat0, 32, 16), 16, v(w.da1, 32), D, grad, s);
  // s0 = leaky(conv3(a0)) also feeds c0
  check(net::down2_dgrad(v(w.da1, 32), 32, w.wt[DOWN1], 16, v(w.dcat0, 32, 16), D, 1, s, v(w.cat0, 32, 16), 16),
        "down2 grad");
  weight_grad(w, E0B, v(w.a0, 16), 16, v(w.dcat0, 32, 16), D, grad, s);
  // a0 = leaky(conv3(x))
  conv_dgrad(w, E0B, v(w.dcat0, 32, 16), v(w.da0, 16), D, s, v(w.a0, 16), 16);
  weight_grad(w, E0A, v(w.x, 8), 8, v(w.da0, 16), D, grad, s);
}

uint64_t splitmix(uint64_t& state) {
  uint64_t z = (state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

lpc_status sync_flags(int* flags, hipStream_t s) {
  int h[4] = {0, 0, 0, 0};
  check(hipMemcpyAsync(h, flags, sizeof(h), hipMemcpyDeviceToHost, s), "hipMemcpyAsync(flags)");
  check(hipStreamSynchronize(s), "hipStreamSynchronize");
  if (h[0]) return fail(LPC_ERR_INVALID_ARG, "a particle id is outside the lattice");
  return LPC_OK;
}

}  // namespace

extern "C" {

int64_t lpc_net_param_count(void) { return param_count(); }

lpc_status lpc_net_init(float* params, uint64_t seed) {
  if (!params) return fail(LPC_ERR_INVALID_ARG, "params is NULL");
  uint64_t st = seed;
  for (int l = 0; l < kNumLayers; ++l) {
    const LayerDef& L = kLayers[l];
    float* W = params + layer_offset(l);
    const double a = std::sqrt(6.0 / (taps(L.kind) * L.cin)) * (l == OUT ? 0.1 : 1.0);
    for (int64_t i = 0; i < weight_count(L); ++i) {
      const double u = (static_cast<double>(splitmix(st) >> 11) + 0.5) * 0x1.0p-53;
      W[i] = static_cast<float>((2.0 * u - 1.0) * a);
    }
    for (int o = 0; o < L.cout; ++o) W[weight_count(L) + o] = 0.f;
  }
  return LPC_OK;
}

size_t lpc_net_workspace_bytes(int32_t n_side) { return size_ok(n_side) ? layout(nullptr, n_side).total : 0; }

lpc_status lpc_net_features(const lpc_geometry* geom, const float* pos, const int32_t* id, int64_t n,
                            const float* ref_pos, const float* psi1, float* out, void* ws, size_t ws_bytes,
                            void* stream) {
  if (!geom || !pos || !id || !out) return fail(LPC_ERR_INVALID_ARG, "NULL argument");
  if (ref_pos && psi1) return fail(LPC_ERR_INVALID_ARG, "give ref_pos (a target grid) or psi1 (an input grid), not both");
  if (!(geom->box > 0.0) || !std::isfinite(geom->box)) return fail(LPC_ERR_INVALID_ARG, "box must be positive");
  if (n < 1 || n > (int64_t(1) << 31) - 1) return fail(LPC_ERR_INVALID_ARG, "n must be in [1, 2^31 - 1]");
  NetWs w;
  if (lpc_status st = check_net_ws(geom->n_side, ws, ws_bytes, &w)) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  return guarded([&]() {
    check(hipMemsetAsync(w.flags, 0, 4 * sizeof(int), s), "hipMemsetAsync");
    check(net::features(pos, id, n, ref_pos, psi1, geom->n_side, geom->box, out, w.flags, s), "features");
    return sync_flags(w.flags, s);
  });
}

lpc_status lpc_net_forward(int32_t n_side, const float* params, const float* feat, float* out, void* ws,
                           size_t ws_bytes, void* stream) {
  if (!params || !feat || !out) return fail(LPC_ERR_INVALID_ARG, "NULL argument");
  if (lpc_status st = check_params(params)) return st;
  NetWs w;
  if (lpc_status st = check_net_ws(n_side, ws, ws_bytes, &w)) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  return guarded([&]() {
    const size_t V = static_cast<size_t>(n_side) * n_side * n_side;
    check(hipMemcpyAsync(w.feat, feat, V * net::kInputChannels * sizeof(float), hipMemcpyDeviceToDevice, s),
          "copy features");
    forward(w, params, s);
    check(hipMemcpyAsync(out, w.out, V * 3 * sizeof(float), hipMemcpyDeviceToDevice, s), "copy output");
    check(hipStreamSynchronize(s), "hipStreamSynchronize");
    return LPC_OK;
  });
}

lpc_status lpc_net_loss_grad(int32_t n_side, const float* params, const float* feat, const float* target,
                             float* grad, double* loss, void* ws, size_t ws_bytes, void* stream) {
  if (!params || !feat || !target || !grad || !loss) return fail(LPC_ERR_INVALID_ARG, "NULL argument");
  if (lpc_status st = check_params(params)) return st;
  NetWs w;
  if (lpc_status st = check_net_ws(n_side, ws, ws_bytes, &w)) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  return guarded([&]() {
    const int V = n_side * n_side * n_side;
    check(hipMemcpyAsync(w.feat, feat, static_cast<size_t>(V) * net::kInputChannels * sizeof(float),
                         hipMemcpyDeviceToDevice, s),
          "copy features");
    forward(w, params, s);
    backward(w, params, target, grad, s);
    std::vector<double> part(static_cast<size_t>(net::loss_blocks(V)));
    check(hipMemcpyAsync(part.data(), w.loss_part, part.size() * sizeof(double), hipMemcpyDeviceToHost, s),
          "copy loss");
    check(hipStreamSynchronize(s), "hipStreamSynchronize");
    double sum = 0.0;
    for (double p : part) sum += p;
    *loss = sum / (3.0 * V);
    return LPC_OK;
  });
}

lpc_status lpc_net_adam(float* params, float* m, float* v, const float* grad, int64_t step, float lr, void* stream) {
  if (!params || !m || !v || !grad) return fail(LPC_ERR_INVALID_ARG, "NULL argument");
  if (step < 1) return fail(LPC_ERR_INVALID_ARG, "step counts from 1");
  if (!(lr >= 0.f) || !std::isfinite(lr)) return fail(LPC_ERR_INVALID_ARG, "lr must be finite and >= 0");
  hipStream_t s = static_cast<hipStream_t>(stream);
  return guarded([&]() {
    check(net::adam(params, m, v, grad, param_count(), lr, 0.9, 0.999, 1e-8f, step, s), "adam");
    check(hipStreamSynchronize(s), "hipStreamSynchronize");
    return LPC_OK;
  });
}

lpc_status lpc_net_scale_output(float* params, float gain, void* stream) {
  if (!params) return fail(LPC_ERR_INVALID_ARG, "NULL argument");
  if (lpc_status st = check_params(params)) return st;
  if (!std::isfinite(gain)) return fail(LPC_ERR_INVALID_ARG, "gain must be finite");
  hipStream_t s = static_cast<hipStream_t>(stream);
  return guarded([&]() {
    // the output layer's weights and biases are the last block of the parameter vector
    check(net::scale(params + layer_offset(OUT), param_count() - layer_offset(OUT), gain, s), "scale");
    return LPC_OK;
  });
}

lpc_status lpc_net_symmetry(int32_t n_side, int32_t k, int32_t channels, const float* in, float* out, void* stream) {
  if (!in || !out) return fail(LPC_ERR_INVALID_ARG, "NULL argument");
  if (n_side < 1 || n_side > 1024) return fail(LPC_ERR_INVALID_ARG, "n_side must be in [1, 1024]");
  if (k < 0 || k >= 48) return fail(LPC_ERR_INVALID_ARG, "k must be in [0, 48)");
  if (channels < 3 || channels > 48 || channels % 3 != 0)
    return fail(LPC_ERR_INVALID_ARG, "channels must be a multiple of 3 in [3, 48]");
  const size_t bytes = static_cast<size_t>(n_side) * n_side * n_side * channels * sizeof(float);
  const char *a = reinterpret_cast<const char*>(in), *b = reinterpret_cast<const char*>(out);
  if (a < b + bytes && b < a + bytes) return fail(LPC_ERR_INVALID_ARG, "out overlaps in");
  hipStream_t s = static_cast<hipStream_t>(stream);
  return guarded([&]() {
    check(net::symmetry(in, out, n_side, channels, k, s), "symmetry");
    return LPC_OK;
  });
}

lpc_status lpc_net_apply(const lpc_geometry* geom, const float* params, const lpc_particles* inout, void* ws,
                         size_t ws_bytes, void* stream) {
  if (!geom || !params || !inout || !inout->pos || !inout->psi1 || !inout->id)
    return fail(LPC_ERR_INVALID_ARG, "NULL argument (params, pos, psi1 and id are needed)");
  if (!(geom->box > 0.0) || !std::isfinite(geom->box)) return fail(LPC_ERR_INVALID_ARG, "box must be positive");
  if (lpc_status st = check_params(params)) return st;
  const int N = geom->n_side;
  NetWs w;
  if (lpc_status st = check_net_ws(N, ws, ws_bytes, &w)) return st;
  const int64_t V = static_cast<int64_t>(N) * N * N;
  if (inout->n != V) return fail(LPC_ERR_INVALID_ARG, "particles.n must equal n_side^3 (one particle per lattice site)");
  hipStream_t s = static_cast<hipStream_t>(stream);
  return guarded([&]() {
    check(hipMemsetAsync(w.flags, 0, 4 * sizeof(int), s), "hipMemsetAsync");
    check(hipMemsetAsync(w.x, 0, static_cast<size_t>(V) * 8 * sizeof(bf16), s), "hipMemsetAsync");
    check(net::features_packed(inout->pos, inout->id, inout->n, inout->psi1, N, geom->box, w.x, w.flags, s),
          "features");
    forward(w, params, s, true);
    check(net::apply_residual(inout->pos, inout->id, inout->n, w.out, N, geom->box, w.flags, s), "apply");
    return sync_flags(w.flags, s);
  });
}

}  // extern "C"
