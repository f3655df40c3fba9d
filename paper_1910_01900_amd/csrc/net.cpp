// Learned coarse-grid correction: the network handle, its workspace layout,
// forward and backward passes and the Adam training step (kernels in
// net_kernels.hip).
#include <cmath>
#include <cstring>
#include <vector>

#include "net_internal.h"

using namespace hmg;

namespace {

constexpr int kChunk = 16;  // bricks (of 64 points) per weight-gradient chunk
constexpr int kLossParts = 256;

int pad16(int x) { return (x + 15) / 16 * 16; }
size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

// activation / gradient buffer ids
enum Act { A0, A1, P1, A2, P2, A3, P3, A4, U3, A5, U2, A6, U1, OUT, NACT };

struct BufSpec {
  int level, ch;
};
const BufSpec kBuf[NACT] = {{0, 16}, {0, 16}, {1, 16}, {1, 32}, {2, 32}, {2, 48}, {3, 48},
                            {3, 48}, {2, 48}, {2, 32}, {1, 32}, {1, 16}, {0, 16}, {0, 1}};

// SplitMix64 (Steele, Lea, Flood 2014)
uint64_t splitmix(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

int64_t points(const hmg_net* N, int batch, int level) {
  const int64_t g = N->G >> level;
  return (int64_t)batch * g * g * g;
}
float* act(const hmg_net* N, int i) { return N->f(N->off_act[i]); }
float* grd(const hmg_net* N, int i) { return N->f(N->off_grad[i]); }

int prep_weights(hmg_net* N, hipStream_t s) {
  if (!N->dirty) return HMG_OK;
  for (auto& l : N->L)
    TRY(net_weight_prep(N->f(N->off_w) + l.off_w, l.cin, l.cout, (uint16_t*)(N->ws + l.off_wf), l.cout_pad, l.kpad_f,
                        (uint16_t*)(N->ws + l.off_wt), l.cin_pad, l.kpad_t, s));
  N->dirty = false;
  return HMG_OK;
}

int conv(const hmg_net* N, int li, const float* x, float* y, int batch, hipStream_t s) {
  const NetLayer& l = N->L[li];
  ConvArgs a;
  a.x = x;
  a.w = (const uint16_t*)(N->ws + l.off_wf);
  a.bias = N->f(N->off_w) + l.off_b;
  a.y = y;
  a.P = (int)points(N, batch, l.level);
  a.g = N->G >> l.level;
  a.cin = l.cin;
  a.cout = l.cout;
  a.cout_pad = l.cout_pad;
  a.kpad = l.kpad_f;
  a.relu = l.relu;
  a.accumulate = 0;
  return net_conv(a, s);
}

// dx = (d/dx of layer li)^T dz: a convolution of dz with the flipped,
// transposed weights.
int conv_t(const hmg_net* N, int li, const float* dz, float* dx, int batch, hipStream_t s) {
  const NetLayer& l = N->L[li];
  ConvArgs a;
  a.x = dz;
  a.w = (const uint16_t*)(N->ws + l.off_wt);
  a.bias = nullptr;
  a.y = dx;
  a.P = (int)points(N, batch, l.level);
  a.g = N->G >> l.level;
  a.cin = l.cout;
  a.cout = l.cin;
  a.cout_pad = l.cin_pad;
  a.kpad = l.kpad_t;
  a.relu = 0;
  a.accumulate = 0;
  return net_conv(a, s);
}

int wgrad(const hmg_net* N, int li, const float* x, const float* dz, int batch, hipStream_t s) {
  const NetLayer& l = N->L[li];
  WgradArgs a;
  a.x = x;
  a.dz = dz;
  a.part = N->f(N->off_part);
  a.bpart = N->f(N->off_bpart);
  a.P = (int)points(N, batch, l.level);
  a.g = N->G >> l.level;
  a.cin = l.cin;
  a.cout = l.cout;
  a.cout_pad = l.cout_pad;
  a.kpad = l.kpad_f;
  a.chunk = kChunk;
  a.nchunk = (int)((net_bricks(batch, a.g) + kChunk - 1) / kChunk);
  return net_wgrad(a, N->f(N->off_g) + l.off_w, N->f(N->off_g) + l.off_b, s);
}

int relu_bwd(const hmg_net* N, int buf, int batch, hipStream_t s) {
  const int64_t n = points(N, batch, kBuf[buf].level) * kBuf[buf].ch;
  return net_relu_bwd(act(N, buf), grd(N, buf), grd(N, buf), n, s);
}

}  // namespace

namespace hmg {

int net_prepare(hmg_net* N, hipStream_t s) { return prep_weights(N, s); }

int net_forward(hmg_net* N, const float* in, float* out, int batch, hipStream_t s) {
  TRY(prep_weights(N, s));
  const int G = N->G;
  TRY(conv(N, 0, in, act(N, A0), batch, s));
  TRY(conv(N, 1, act(N, A0), act(N, A1), batch, s));
  TRY(net_pool(act(N, A1), act(N, P1), batch, G, 16, s));
  TRY(conv(N, 2, act(N, P1), act(N, A2), batch, s));
  TRY(net_pool(act(N, A2), act(N, P2), batch, G / 2, 32, s));
  TRY(conv(N, 3, act(N, P2), act(N, A3), batch, s));
  TRY(net_pool(act(N, A3), act(N, P3), batch, G / 4, 48, s));
  TRY(conv(N, 4, act(N, P3), act(N, A4), batch, s));
  TRY(net_up_add(act(N, A4), act(N, A3), act(N, U3), batch, G / 4, 48, s));
  TRY(conv(N, 5, act(N, U3), act(N, A5), batch, s));
  TRY(net_up_add(act(N, A5), act(N, A2), act(N, U2), batch, G / 2, 32, s));
  TRY(conv(N, 6, act(N, U2), act(N, A6), batch, s));
  TRY(net_up_add(act(N, A6), act(N, A1), act(N, U1), batch, G, 16, s));
  return conv(N, 7, act(N, U1), out, batch, s);
}

}  // namespace hmg

namespace {

// Masked MSE of out against tgt and every parameter gradient (into the
// gradient vector); the forward pass must have run on `in`.
int loss_and_grad(hmg_net* N, const float* in, const float* tgt, int batch, double* loss, hipStream_t s) {
  const int G = N->G;
  const int g3 = G * G * G;
  double* lpart = (double*)(N->ws + N->off_lpart);
  TRY(net_mse(act(N, OUT), tgt, in, batch, g3, grd(N, OUT), lpart, kLossParts, loss, s));
  TRY(wgrad(N, 7, act(N, U1), grd(N, OUT), batch, s));
  TRY(conv_t(N, 7, grd(N, OUT), grd(N, U1), batch, s));
  TRY(net_up_bwd(grd(N, U1), grd(N, A6), batch, G, 16, s));
  TRY(relu_bwd(N, A6, batch, s));
  TRY(wgrad(N, 6, act(N, U2), grd(N, A6), batch, s));
  TRY(conv_t(N, 6, grd(N, A6), grd(N, U2), batch, s));
  TRY(net_up_bwd(grd(N, U2), grd(N, A5), batch, G / 2, 32, s));
  TRY(relu_bwd(N, A5, batch, s));
  TRY(wgrad(N, 5, act(N, U3), grd(N, A5), batch, s));
  TRY(conv_t(N, 5, grd(N, A5), grd(N, U3), batch, s));
  TRY(net_up_bwd(grd(N, U3), grd(N, A4), batch, G / 4, 48, s));
  TRY(relu_bwd(N, A4, batch, s));
  TRY(wgrad(N, 4, act(N, P3), grd(N, A4), batch, s));
  TRY(conv_t(N, 4, grd(N, A4), grd(N, P3), batch, s));
  // level G/4: skip gradient from U3 plus the pooled path
  TRY(net_copy(grd(N, U3), grd(N, A3), points(N, batch, 2) * 48, s));
  TRY(net_pool_bwd(grd(N, P3), grd(N, A3), batch, G / 4, 48, 1, s));
  TRY(relu_bwd(N, A3, batch, s));
  TRY(wgrad(N, 3, act(N, P2), grd(N, A3), batch, s));
  TRY(conv_t(N, 3, grd(N, A3), grd(N, P2), batch, s));
  TRY(net_copy(grd(N, U2), grd(N, A2), points(N, batch, 1) * 32, s));
  TRY(net_pool_bwd(grd(N, P2), grd(N, A2), batch, G / 2, 32, 1, s));
  TRY(relu_bwd(N, A2, batch, s));
  TRY(wgrad(N, 2, act(N, P1), grd(N, A2), batch, s));
  TRY(conv_t(N, 2, grd(N, A2), grd(N, P1), batch, s));
  TRY(net_copy(grd(N, U1), grd(N, A1), points(N, batch, 0) * 16, s));
  TRY(net_pool_bwd(grd(N, P1), grd(N, A1), batch, G, 16, 1, s));
  TRY(relu_bwd(N, A1, batch, s));
  TRY(wgrad(N, 1, act(N, A0), grd(N, A1), batch, s));
  TRY(conv_t(N, 1, grd(N, A1), grd(N, A0), batch, s));
  TRY(relu_bwd(N, A0, batch, s));
  return wgrad(N, 0, in, grd(N, A0), batch, s);
}

int check_net(const hmg_net* N) {
  if (!N) return fail(HMG_ERR_INVALID, "network is NULL");
  if (!N->bound) return fail(HMG_ERR_WORKSPACE, "network is not bound to a workspace");
  return HMG_OK;
}

int check_batch_args(const hmg_net* N, const void* in, const void* out, int batch) {
  TRY(check_net(N));
  if (batch < 1 || batch > N->max_batch) return fail(HMG_ERR_INVALID, "batch must be 1..max_batch");
  TRY(check_ptr(in, "input"));
  return check_ptr(out, "output");
}

}  // namespace

extern "C" int hmg_net_create(int grid, int max_batch, uint64_t seed, hmg_net** out) {
  if (!out) return fail(HMG_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (grid < 8 || grid > 64 || grid % 8) return fail(HMG_ERR_INVALID, "grid must be a multiple of 8 in 8..64");
  if (max_batch < 1 || max_batch > 4096) return fail(HMG_ERR_INVALID, "max_batch must be 1..4096");
  if ((int64_t)max_batch * grid * grid * grid * 48 > ((int64_t)1 << 31))
    return fail(HMG_ERR_UNSUPPORTED, "batch too large");
  auto* N = new hmg_net;
  N->G = grid;
  N->max_batch = max_batch;
  N->seed = seed;
  const int spec[kNetLayers][4] = {{2, 16, 0, 1},  {16, 16, 0, 1}, {16, 32, 1, 1}, {32, 48, 2, 1},
                                   {48, 48, 3, 1}, {48, 32, 2, 1}, {32, 16, 1, 1}, {16, 1, 0, 0}};
  int64_t np = 0;
  for (int i = 0; i < kNetLayers; ++i) {
    NetLayer& l = N->L[i];
    l.cin = spec[i][0];
    l.cout = spec[i][1];
    l.level = spec[i][2];
    l.relu = spec[i][3];
    l.off_w = np;
    np += (int64_t)l.cout * 27 * l.cin;
    l.off_b = np;
    np += l.cout;
    l.cout_pad = pad16(l.cout);
    l.kpad_f = pad16(27 * l.cin);
    l.cin_pad = pad16(l.cin);
    l.kpad_t = pad16(27 * l.cout);
  }
  N->n_params = np;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t r = o;
    o = al(o + bytes);
    return r;
  };
  N->off_w = take(np * 4);
  N->off_g = take(np * 4);
  N->off_m = take(np * 4);
  N->off_v = take(np * 4);
  int64_t part = 0;
  for (auto& l : N->L) {
    l.off_wf = take((size_t)l.cout_pad * l.kpad_f * 2);
    l.off_wt = take((size_t)l.cin_pad * l.kpad_t * 2);
    const int64_t nch = (net_bricks(max_batch, N->G >> l.level) + kChunk - 1) / kChunk;
    part = std::max<int64_t>(part, nch * l.cout_pad * l.kpad_f);
  }
  N->part_floats = part;
  N->off_part = take(part * 4);
  N->off_bpart = take((size_t)((points(N, max_batch, 0) + 255) / 256) * 48 * 4);
  for (int i = 0; i < NACT; ++i) {
    const size_t bytes = (size_t)points(N, max_batch, kBuf[i].level) * kBuf[i].ch * 4;
    N->off_act[i] = take(bytes);
    N->off_grad[i] = take(bytes);
  }
  N->off_lpart = take((kLossParts + 1) * 8);
  N->off_loss = take(8);
  const int64_t g3 = (int64_t)grid * grid * grid;
  N->off_hin = take(g3 * 2 * 4);
  N->off_hout = take(g3 * 4);
  N->off_hsig = take(8);
  N->ws_bytes = o;
  *out = N;
  return HMG_OK;
}

extern "C" int hmg_net_query(const hmg_net* N, int64_t* n_params, size_t* ws) {
  if (!N) return fail(HMG_ERR_INVALID, "network is NULL");
  if (n_params) *n_params = N->n_params;
  if (ws) *ws = N->ws_bytes;
  return HMG_OK;
}

extern "C" int hmg_net_bind(hmg_net* N, void* ws, size_t bytes, hipStream_t s) {
  if (!N) return fail(HMG_ERR_INVALID, "network is NULL");
  if (!ws || ((uintptr_t)ws & 255)) return fail(HMG_ERR_WORKSPACE, "workspace NULL or not 256-byte aligned");
  if (bytes < N->ws_bytes) return fail(HMG_ERR_WORKSPACE, "workspace too small");
  N->ws = (char*)ws;
  // He-uniform weights U(-sqrt(6 / fan_in), sqrt(6 / fan_in)), zero biases
  std::vector<float> w((size_t)N->n_params, 0.f);
  uint64_t st = N->seed;
  for (auto& l : N->L) {
    const double a = std::sqrt(6.0 / (27.0 * l.cin));
    for (int64_t i = 0; i < (int64_t)l.cout * 27 * l.cin; ++i) {
      const double u = (double)(splitmix(st) >> 11) * 0x1.0p-53;
      w[(size_t)(l.off_w + i)] = (float)((2.0 * u - 1.0) * a);
    }
  }
  std::vector<float> z((size_t)N->n_params, 0.f);
  HMG_HIP(hipMemcpyAsync(N->f(N->off_w), w.data(), w.size() * 4, hipMemcpyHostToDevice, s));
  HMG_HIP(hipMemcpyAsync(N->f(N->off_m), z.data(), z.size() * 4, hipMemcpyHostToDevice, s));
  HMG_HIP(hipMemcpyAsync(N->f(N->off_v), z.data(), z.size() * 4, hipMemcpyHostToDevice, s));
  HMG_HIP(hipStreamSynchronize(s));
  N->step = 0;
  N->dirty = true;
  N->version++;
  N->bound = true;
  return HMG_OK;
}

extern "C" void hmg_net_destroy(hmg_net* N) { delete N; }

extern "C" int hmg_net_get_params(const hmg_net* N, float* dst, hipStream_t s) {
  TRY(check_net(N));
  TRY(check_ptr(dst, "dst"));
  HMG_HIP(hipMemcpyAsync(dst, N->f(N->off_w), (size_t)N->n_params * 4, hipMemcpyDeviceToDevice, s));
  return HMG_OK;
}

extern "C" int hmg_net_set_params(hmg_net* N, const float* src, hipStream_t s) {
  TRY(check_net(N));
  TRY(check_ptr(src, "src"));
  HMG_HIP(hipMemcpyAsync(N->f(N->off_w), src, (size_t)N->n_params * 4, hipMemcpyDeviceToDevice, s));
  N->dirty = true;
  N->version++;
  return HMG_OK;
}

extern "C" int hmg_net_forward(hmg_net* N, const float* in, float* out, int batch, hipStream_t s) {
  TRY(check_batch_args(N, in, out, batch));
  return net_forward(N, in, out, batch, s);
}

extern "C" int hmg_net_gradient(hmg_net* N, const float* in, const float* target, int batch, float* grad,
                                double* loss, hipStream_t s) {
  TRY(check_batch_args(N, in, target, batch));
  TRY(check_ptr(grad, "grad"));
  TRY(check_ptr(loss, "loss"));
  TRY(net_forward(N, in, act(N, OUT), batch, s));
  TRY(loss_and_grad(N, in, target, batch, loss, s));
  HMG_HIP(hipMemcpyAsync(grad, N->f(N->off_g), (size_t)N->n_params * 4, hipMemcpyDeviceToDevice, s));
  return HMG_OK;
}

extern "C" int hmg_net_train_step(hmg_net* N, const float* in, const float* target, int batch, double lr,
                                  double* loss, hipStream_t s) {
  TRY(check_batch_args(N, in, target, batch));
  if (!(lr > 0)) return fail(HMG_ERR_INVALID, "lr must be positive");
  TRY(net_forward(N, in, act(N, OUT), batch, s));
  double* dl = loss ? loss : (double*)(N->ws + N->off_loss);
  TRY(loss_and_grad(N, in, target, batch, dl, s));
  const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
  N->step++;
  const double lr_t = lr * std::sqrt(1.0 - std::pow(b2, (double)N->step)) / (1.0 - std::pow(b1, (double)N->step));
  TRY(net_adam(N->f(N->off_w), N->f(N->off_g), N->f(N->off_m), N->f(N->off_v), N->n_params, (float)lr_t, (float)b1,
               (float)b2, (float)eps, s));
  N->dirty = true;
  N->version++;
  return HMG_OK;
}
