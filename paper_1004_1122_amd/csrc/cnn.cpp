// Warm-start network: parameter layout, forward and backward sequencing, and
// the C ABI of include/lshom_cnn.h.  Every arithmetic step runs in the
// kernels of cnn_kernels.hip; this file only plans buffers and launches.
#include "lshom_cnn.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "cnn.hpp"

using namespace lshom::cnn;

namespace {

enum Kind { K_CONV3 = 0, K_DOWN3 = 1, K_CONV1 = 2 };

struct Layer {
  std::string name;
  int kind;
  int cin;        // channels the kernel reads (input layer: 8, two of them real)
  int cin_real;   // channels of the compact parameter order
  int cout;       // real output channels
  int np;         // output channels padded to a multiple of 8
  int taps;
  size_t w_off, b_off;  // offsets (elements) into the parameter arrays
};

constexpr size_t kAlignEl = 64;  // parameter blocks start on 256-byte boundaries
size_t align_el(size_t v) { return (v + kAlignEl - 1) / kAlignEl * kAlignEl; }
size_t align_b(size_t v) { return (v + 255) / 256 * 256; }
int pad8(int c) { return (c + 7) / 8 * 8; }

}  // namespace

struct lshom_cnn {
  int device = 0;
  hipStream_t user_stream = nullptr, stream = nullptr;
  hipEvent_t ev = nullptr;
  std::string err;
  int c0 = 32;
  std::vector<Layer> layers;
  size_t n_el = 0;         // elements per parameter array (padded layout)
  long long n_compact = 0;
  // parameter buffer
  char* pbuf = nullptr;
  size_t pbytes = 0;
  float *w = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
  bf16_t *w16 = nullptr, *wt16 = nullptr;
  int adam_t = 0;
  bool params_set = false;
  // workspace
  char* ws = nullptr;
  size_t ws_bytes = 0;
  int ws_B = 0, ws_N = 0, ws_train = 0;
};

namespace {

lshom_status fail(lshom_cnn* c, lshom_status s, const std::string& m) {
  if (c) c->err = m;
  return s;
}

#define CNN_TRY(ctx, expr)                                                                        \
  do {                                                                                            \
    hipError_t e_ = (expr);                                                                       \
    if (e_ != hipSuccess) return fail((ctx), LSHOM_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

void build_layers(lshom_cnn* c) {
  const int c0 = c->c0;
  const int w[4] = {c0, 2 * c0, 4 * c0, 8 * c0};
  auto add = [&](const char* name, int kind, int cin, int cin_real, int cout) {
    Layer L;
    L.name = name;
    L.kind = kind;
    L.cin = cin;
    L.cin_real = cin_real;
    L.cout = cout;
    L.np = pad8(cout);
    L.taps = kind == K_CONV1 ? 1 : 9;
    c->layers.push_back(L);
  };
  add("enc0a", K_CONV3, 8, 2, w[0]);
  add("enc0b", K_CONV3, w[0], w[0], w[0]);
  add("down0", K_DOWN3, w[0], w[0], w[1]);
  add("enc1a", K_CONV3, w[1], w[1], w[1]);
  add("enc1b", K_CONV3, w[1], w[1], w[1]);
  add("down1", K_DOWN3, w[1], w[1], w[2]);
  add("enc2a", K_CONV3, w[2], w[2], w[2]);
  add("enc2b", K_CONV3, w[2], w[2], w[2]);
  add("down2", K_DOWN3, w[2], w[2], w[3]);
  add("bot_a", K_CONV3, w[3], w[3], w[3]);
  add("bot_b", K_CONV3, w[3], w[3], w[3]);
  for (int lev = 2; lev >= 0; --lev) {
    const std::string s = std::to_string(lev);
    add(("up" + s).c_str(), K_CONV3, w[lev + 1], w[lev + 1], w[lev]);
    add(("dec" + s + "a").c_str(), K_CONV3, 2 * w[lev], 2 * w[lev], w[lev]);
    add(("dec" + s + "b").c_str(), K_CONV3, w[lev], w[lev], w[lev]);
  }
  add("head", K_CONV1, w[0], w[0], 2);
  size_t off = 0;
  long long compact = 0;
  for (Layer& L : c->layers) {
    L.w_off = off;
    off = align_el(off + (size_t)L.taps * L.cin * L.np);
    L.b_off = off;
    off = align_el(off + (size_t)L.np);
    compact += (long long)L.taps * L.cin_real * L.cout + L.cout;
  }
  c->n_el = off;
  c->n_compact = compact;
}

const Layer& layer(const lshom_cnn* c, const char* name) {
  for (const Layer& L : c->layers)
    if (L.name == name) return L;
  return c->layers[0];
}

// Workspace plan for (B, N, training).
struct Plan {
  size_t total = 0;
  long long P[4];
  int Nl[4];
  // forward (bf16 element offsets into bytes)
  size_t x, enc0a, cat0, down0, enc1a, cat1, down1, enc2a, cat2, down2, bota, botb, dec2a, dec2b, dec1a, dec1b,
      dec0a, dec0b, out;
  // training
  size_t gout, gpre, gA, gB, dcat0, dcat1, dcat2, partial, part, loss;
  size_t partial_floats = 0;
};

int splits_for(long long P) {
  long long s = (P + 8191) / 8192;
  return (int)std::max(1LL, std::min(64LL, s));
}

Plan make_plan(const lshom_cnn* c, int B, int N, int training) {
  Plan p;
  for (int l = 0, n = N; l < 4; ++l, n /= 3) {
    p.Nl[l] = n;
    p.P[l] = (long long)B * n * n;
  }
  const int c0 = c->c0;
  size_t off = 0;
  auto bf = [&](long long pix, int ch) {
    const size_t o = off;
    off = align_b(off + (size_t)pix * ch * 2);
    return o;
  };
  auto f32 = [&](long long count) {
    const size_t o = off;
    off = align_b(off + (size_t)count * 4);
    return o;
  };
  p.x = bf(p.P[0], 8);
  p.enc0a = bf(p.P[0], c0);
  p.cat0 = bf(p.P[0], 2 * c0);
  p.down0 = bf(p.P[1], 2 * c0);
  p.enc1a = bf(p.P[1], 2 * c0);
  p.cat1 = bf(p.P[1], 4 * c0);
  p.down1 = bf(p.P[2], 4 * c0);
  p.enc2a = bf(p.P[2], 4 * c0);
  p.cat2 = bf(p.P[2], 8 * c0);
  p.down2 = bf(p.P[3], 8 * c0);
  p.bota = bf(p.P[3], 8 * c0);
  p.botb = bf(p.P[3], 8 * c0);
  p.dec2a = bf(p.P[2], 4 * c0);
  p.dec2b = bf(p.P[2], 4 * c0);
  p.dec1a = bf(p.P[1], 2 * c0);
  p.dec1b = bf(p.P[1], 2 * c0);
  p.dec0a = bf(p.P[0], c0);
  p.dec0b = bf(p.P[0], c0);
  p.out = f32(p.P[0] * 2);
  if (training) {
    p.gout = f32(p.P[0] * 2);
    long long gmax = 0;
    for (int l = 0; l < 4; ++l) gmax = std::max(gmax, p.P[l] * (long long)(c0 << l));
    p.gpre = bf(gmax > p.P[0] * 8 ? gmax : p.P[0] * 8, 1);
    long long gab = 0;
    for (int l = 0; l < 4; ++l) gab = std::max(gab, p.P[l] * (long long)(2 * c0 << l));
    p.gA = f32(gab);
    p.gB = f32(gab);
    p.dcat0 = f32(p.P[0] * 2 * c0);
    p.dcat1 = f32(p.P[1] * 4 * c0);
    p.dcat2 = f32(p.P[2] * 8 * c0);
    size_t pf = 0;
    const int lev_of[] = {0, 0, 1, 1, 1, 2, 2, 2, 3, 3, 3, 2, 2, 2, 1, 1, 1, 0, 0, 0, 0};
    for (size_t i = 0; i < c->layers.size(); ++i) {
      const Layer& L = c->layers[i];
      const long long Pout = p.P[lev_of[i]];
      const size_t rows = (size_t)L.taps * L.cin + 1;
      pf = std::max(pf, (size_t)splits_for(Pout) * rows * L.np);
    }
    p.partial_floats = pf;
    p.partial = f32((long long)pf);
    p.part = f32(2LL * B * 256 * 2);  // doubles
    p.loss = f32(2);
  }
  p.total = off;
  return p;
}

template <typename T>
T* at(lshom_cnn* c, size_t off) {
  return reinterpret_cast<T*>(c->ws + off);
}

hipError_t order_after_user(lshom_cnn* c) {
  hipError_t e = hipEventRecord(c->ev, c->user_stream);
  if (e != hipSuccess) return e;
  return hipStreamWaitEvent(c->stream, c->ev, 0);
}

// --- launch helpers --------------------------------------------------------

struct View {
  const bf16_t* p;
  int C, ld;
};

hipError_t conv_fwd(lshom_cnn* c, const Layer& L, View in, int B, int Hi, int Ho, int mode, int up, bf16_t* out_b,
                    int ldb, float* out_f, int ldf, bool relu) {
  ConvArgs a{};
  a.in0 = in.p;
  a.C0 = in.C;
  a.ld0 = in.ld;
  a.in1 = nullptr;
  a.C1 = 0;
  a.ld1 = 0;
  a.B = B;
  a.Hi = a.Wi = Hi;
  a.Ho = a.Wo = Ho;
  a.mode = mode;
  a.up = up;
  a.w = c->w16 + L.w_off;
  a.ldw = L.taps * L.cin;
  a.N = L.cout;
  a.Np = L.np;
  a.bias = c->w + L.b_off;
  a.relu = relu ? 1 : 0;
  a.out_b = out_b;
  a.ldb = ldb;
  a.out_f = out_f;
  a.ldf = ldf;
  a.accumulate = 0;
  return launch_conv(a, c->stream);
}

// input gradient of layer L: gpre [Pout][np] -> out_f [Pin][cin]
hipError_t conv_dgrad(lshom_cnn* c, const Layer& L, const bf16_t* gpre, int B, int Hout, float* out_f) {
  ConvArgs a{};
  a.in0 = gpre;
  a.C0 = L.np;
  a.ld0 = L.np;
  a.B = B;
  a.w = c->wt16 + L.w_off;
  a.ldw = L.taps * L.np;
  a.N = L.cin;
  a.Np = L.cin;
  a.bias = nullptr;
  a.relu = 0;
  a.out_f = out_f;
  a.ldf = L.cin;
  a.accumulate = 0;
  if (L.kind == K_CONV3) {
    a.mode = CM_CONV3;
    a.up = 1;
    a.Hi = a.Wi = a.Ho = a.Wo = Hout;
  } else if (L.kind == K_DOWN3) {
    a.mode = CM_DOWN3_T;
    a.up = 1;
    a.Hi = a.Wi = a.Ho = a.Wo = Hout;  // coarse grid; output on the 3x finer one
  } else {
    a.mode = CM_POINT;
    a.up = 1;
    a.Hi = a.Wi = a.Ho = a.Wo = Hout;
  }
  return launch_conv(a, c->stream);
}

hipError_t conv_wgrad(lshom_cnn* c, const Plan& p, const Layer& L, View in, int B, int Hi, int Ho, int mode, int up,
                      const bf16_t* gpre) {
  WgradArgs a{};
  a.in0 = in.p;
  a.C0 = in.C;
  a.ld0 = in.ld;
  a.in1 = nullptr;
  a.C1 = 0;
  a.ld1 = 0;
  a.B = B;
  a.Hi = a.Wi = Hi;
  a.Ho = a.Wo = Ho;
  a.mode = mode;
  a.up = up;
  a.gy = gpre;
  a.ldg = L.np;
  a.Np = L.np;
  a.taps = L.taps;
  a.rows = L.taps * L.cin + 1;
  const long long P = (long long)B * Ho * Ho;
  const int splits = splits_for(P);
  long long pps = (P + splits - 1) / splits;
  pps = (pps + 31) / 32 * 32;
  a.pix_per_split = pps;
  float* partial = at<float>(c, p.partial);
  a.partial = partial;
  hipError_t e = launch_wgrad(a, splits, c->stream);
  if (e != hipSuccess) return e;
  return launch_wgrad_reduce(partial, splits, a.rows, L.np, c->g + L.w_off, c->g + L.b_off, c->stream);
}

hipError_t prep(lshom_cnn* c, long long P, int C, int Cp, const float* g0, int ld0, const float* g1, int ld1,
                const bf16_t* act, int lda, bf16_t* gpre) {
  return launch_grad_prep(P, C, Cp, g0, ld0, g1, ld1, act, lda, gpre, c->stream);
}

hipError_t cast_all(lshom_cnn* c) {
  for (const Layer& L : c->layers) {
    hipError_t e = launch_cast_weights(c->w + L.w_off, L.taps, L.cin, L.np, L.kind == K_CONV3 ? 1 : 0,
                                       c->w16 + L.w_off, c->wt16 + L.w_off, c->stream);
    if (e != hipSuccess) return e;
    // bias copies are read in FP32; nothing to cast
  }
  return hipSuccess;
}

// --- forward and backward ----------------------------------------------------

hipError_t forward(lshom_cnn* c, const Plan& p, int B, const uint8_t* phase, const float* lr, int transpose,
                   int scale) {
  const int c0 = c->c0;
  const int* Nl = p.Nl;
  hipError_t e;
  bf16_t* x = at<bf16_t>(c, p.x);
#define FWD(expr)                          \
  if ((e = (expr)) != hipSuccess) return e
  FWD(launch_make_input(B, Nl[0], phase, lr, transpose, scale, x, c->stream));
  bf16_t* cat0 = at<bf16_t>(c, p.cat0);
  bf16_t* cat1 = at<bf16_t>(c, p.cat1);
  bf16_t* cat2 = at<bf16_t>(c, p.cat2);
  FWD(conv_fwd(c, layer(c, "enc0a"), View{x, 8, 8}, B, Nl[0], Nl[0], CM_CONV3, 1, at<bf16_t>(c, p.enc0a), c0, nullptr,
               0, true));
  FWD(conv_fwd(c, layer(c, "enc0b"), View{at<bf16_t>(c, p.enc0a), c0, c0}, B, Nl[0], Nl[0], CM_CONV3, 1, cat0 + c0,
               2 * c0, nullptr, 0, true));
  FWD(conv_fwd(c, layer(c, "down0"), View{cat0 + c0, c0, 2 * c0}, B, Nl[0], Nl[1], CM_DOWN3, 1,
               at<bf16_t>(c, p.down0), 2 * c0, nullptr, 0, true));
  FWD(conv_fwd(c, layer(c, "enc1a"), View{at<bf16_t>(c, p.down0), 2 * c0, 2 * c0}, B, Nl[1], Nl[1], CM_CONV3, 1,
               at<bf16_t>(c, p.enc1a), 2 * c0, nullptr, 0, true));
  FWD(conv_fwd(c, layer(c, "enc1b"), View{at<bf16_t>(c, p.enc1a), 2 * c0, 2 * c0}, B, Nl[1], Nl[1], CM_CONV3, 1,
               cat1 + 2 * c0, 4 * c0, nullptr, 0, true));
  FWD(conv_fwd(c, layer(c, "down1"), View{cat1 + 2 * c0, 2 * c0, 4 * c0}, B, Nl[1], Nl[2], CM_DOWN3, 1,
               at<bf16_t>(c, p.down1), 4 * c0, nullptr, 0, true));
  FWD(conv_fwd(c, layer(c, "enc2a"), View{at<bf16_t>(c, p.down1), 4 * c0, 4 * c0}, B, Nl[2], Nl[2], CM_CONV3, 1,
               at<bf16_t>(c, p.enc2a), 4 * c0, nullptr, 0, true));
  FWD(conv_fwd(c, layer(c, "enc2b"), View{at<bf16_t>(c, p.enc2a), 4 * c0, 4 * c0}, B, Nl[2], Nl[2], CM_CONV3, 1,
               cat2 + 4 * c0, 8 * c0, nullptr, 0, true));
  FWD(conv_fwd(c, layer(c, "down2"), View{cat2 + 4 * c0, 4 * c0, 8 * c0}, B, Nl[2], Nl[3], CM_DOWN3, 1,
               at<bf16_t>(c, p.down2), 8 * c0, nullptr, 0, true));
  FWD(conv_fwd(c, layer(c, "bot_a"), View{at<bf16_t>(c, p.down2), 8 * c0, 8 * c0}, B, Nl[3], Nl[3], CM_CONV3, 1,
               at<bf16_t>(c, p.bota), 8 * c0, nullptr, 0, true));
  FWD(conv_fwd(c, layer(c, "bot_b"), View{at<bf16_t>(c, p.bota), 8 * c0, 8 * c0}, B, Nl[3], Nl[3], CM_CONV3, 1,
               at<bf16_t>(c, p.botb), 8 * c0, nullptr, 0, true));
  // up path: level 2
  FWD(conv_fwd(c, layer(c, "up2"), View{at<bf16_t>(c, p.botb), 8 * c0, 8 * c0}, B, Nl[3], Nl[2], CM_CONV3, 3, cat2,
               8 * c0, nullptr, 0, true));
  FWD(conv_fwd(c, layer(c, "dec2a"), View{cat2, 8 * c0, 8 * c0}, B, Nl[2], Nl[2], CM_CONV3, 1,
               at<bf16_t>(c, p.dec2a), 4 * c0, nullptr, 0, true));
  FWD(conv_fwd(c, layer(c, "dec2b"), View{at<bf16_t>(c, p.dec2a), 4 * c0, 4 * c0}, B, Nl[2], Nl[2], CM_CONV3, 1,
               at<bf16_t>(c, p.dec2b), 4 * c0, nullptr, 0, true));
  // level 1
  FWD(conv_fwd(c, layer(c, "up1"), View{at<bf16_t>(c, p.dec2b), 4 * c0, 4 * c0}, B, Nl[2], Nl[1], CM_CONV3, 3, cat1,
               4 * c0, nullptr, 0, true));
  FWD(conv_fwd(c, layer(c, "dec1a"), View{cat1, 4 * c0, 4 * c0}, B, Nl[1], Nl[1], CM_CONV3, 1,
               at<bf16_t>(c, p.dec1a), 2 * c0, nullptr, 0, true));
  FWD(conv_fwd(c, layer(c, "dec1b"), View{at<bf16_t>(c, p.dec1a), 2 * c0, 2 * c0}, B, Nl[1], Nl[1], CM_CONV3, 1,
               at<bf16_t>(c, p.dec1b), 2 * c0, nullptr, 0, true));
  // level 0
  FWD(conv_fwd(c, layer(c, "up0"), View{at<bf16_t>(c, p.dec1b), 2 * c0, 2 * c0}, B, Nl[1], Nl[0], CM_CONV3, 3, cat0,
               2 * c0, nullptr, 0, true));
  FWD(conv_fwd(c, layer(c, "dec0a"), View{cat0, 2 * c0, 2 * c0}, B, Nl[0], Nl[0], CM_CONV3, 1,
               at<bf16_t>(c, p.dec0a), c0, nullptr, 0, true));
  FWD(conv_fwd(c, layer(c, "dec0b"), View{at<bf16_t>(c, p.dec0a), c0, c0}, B, Nl[0], Nl[0], CM_CONV3, 1,
               at<bf16_t>(c, p.dec0b), c0, nullptr, 0, true));
  FWD(conv_fwd(c, layer(c, "head"), View{at<bf16_t>(c, p.dec0b), c0, c0}, B, Nl[0], Nl[0], CM_POINT, 1, nullptr, 0,
               at<float>(c, p.out), 2, false));
#undef FWD
  return hipSuccess;
}

hipError_t backward(lshom_cnn* c, const Plan& p, int B) {
  const int c0 = c->c0;
  const int* Nl = p.Nl;
  const long long* P = p.P;
  hipError_t e;
#define BWD(expr)                          \
  if ((e = (expr)) != hipSuccess) return e
  bf16_t* gpre = at<bf16_t>(c, p.gpre);
  float* gA = at<float>(c, p.gA);
  float* gB = at<float>(c, p.gB);
  float* dcat0 = at<float>(c, p.dcat0);
  float* dcat1 = at<float>(c, p.dcat1);
  float* dcat2 = at<float>(c, p.dcat2);
  bf16_t* cat0 = at<bf16_t>(c, p.cat0);
  bf16_t* cat1 = at<bf16_t>(c, p.cat1);
  bf16_t* cat2 = at<bf16_t>(c, p.cat2);
  auto A = [&](size_t off) { return at<bf16_t>(c, off); };

  // head (no ReLU)
  {
    const Layer& L = layer(c, "head");
    BWD(prep(c, P[0], 2, L.np, at<float>(c, p.gout), 2, nullptr, 0, nullptr, 0, gpre));
    BWD(conv_wgrad(c, p, L, View{A(p.dec0b), c0, c0}, B, Nl[0], Nl[0], CM_POINT, 1, gpre));
    BWD(conv_dgrad(c, L, gpre, B, Nl[0], gA));
  }
  // one decoder level: dec_b, dec_a, up; returns the coarse gradient in gB
  struct Lev {
    const char *b, *a, *up;
    size_t act_b, act_a, coarse_in;
    bf16_t* cat;
    float* dcat;
    int l;
  };
  const Lev levs[3] = {{"dec0b", "dec0a", "up0", p.dec0b, p.dec0a, p.dec1b, cat0, dcat0, 0},
                       {"dec1b", "dec1a", "up1", p.dec1b, p.dec1a, p.dec2b, cat1, dcat1, 1},
                       {"dec2b", "dec2a", "up2", p.dec2b, p.dec2a, p.botb, cat2, dcat2, 2}};
  for (const Lev& lv : levs) {
    const int l = lv.l;
    const int C = c0 << l;  // channels of this level
    // gradient of dec_b output is in gA (level 0) or gB (after a pool)
    float* g_in = l == 0 ? gA : gB;
    const Layer& Lb = layer(c, lv.b);
    BWD(prep(c, P[l], C, Lb.np, g_in, C, nullptr, 0, A(lv.act_b), C, gpre));
    BWD(conv_wgrad(c, p, Lb, View{A(lv.act_a), C, C}, B, Nl[l], Nl[l], CM_CONV3, 1, gpre));
    float* g_a = l == 0 ? gB : gA;
    BWD(conv_dgrad(c, Lb, gpre, B, Nl[l], g_a));
    const Layer& La = layer(c, lv.a);
    BWD(prep(c, P[l], C, La.np, g_a, C, nullptr, 0, A(lv.act_a), C, gpre));
    BWD(conv_wgrad(c, p, La, View{lv.cat, 2 * C, 2 * C}, B, Nl[l], Nl[l], CM_CONV3, 1, gpre));
    BWD(conv_dgrad(c, La, gpre, B, Nl[l], lv.dcat));
    // up-convolution: output channels [0, C) of the concat buffer
    const Layer& Lu = layer(c, lv.up);
    BWD(prep(c, P[l], C, Lu.np, lv.dcat, 2 * C, nullptr, 0, lv.cat, 2 * C, gpre));
    BWD(conv_wgrad(c, p, Lu, View{A(lv.coarse_in), 2 * C, 2 * C}, B, Nl[l + 1], Nl[l], CM_CONV3, 3, gpre));
    BWD(conv_dgrad(c, Lu, gpre, B, Nl[l], gA));  // fine-grid gradient of the upsampled input
    BWD(launch_pool3_sum(B, Nl[l + 1], Nl[l + 1], 2 * C, gA, gB, c->stream));
  }
  // bottom: gradient of bot_b output in gB
  {
    const int C = 8 * c0;
    const Layer& Lb = layer(c, "bot_b");
    BWD(prep(c, P[3], C, Lb.np, gB, C, nullptr, 0, A(p.botb), C, gpre));
    BWD(conv_wgrad(c, p, Lb, View{A(p.bota), C, C}, B, Nl[3], Nl[3], CM_CONV3, 1, gpre));
    BWD(conv_dgrad(c, Lb, gpre, B, Nl[3], gA));
    const Layer& La = layer(c, "bot_a");
    BWD(prep(c, P[3], C, La.np, gA, C, nullptr, 0, A(p.bota), C, gpre));
    BWD(conv_wgrad(c, p, La, View{A(p.down2), C, C}, B, Nl[3], Nl[3], CM_CONV3, 1, gpre));
    BWD(conv_dgrad(c, La, gpre, B, Nl[3], gB));
  }
  // encoder levels 2, 1, 0: gradient of down_l output in gB
  struct Enc {
    const char *down, *b, *a;
    size_t act_down, act_a, in_a;
    bf16_t* cat;
    float* dcat;
    int l;
  };
  const Enc encs[3] = {{"down2", "enc2b", "enc2a", p.down2, p.enc2a, p.down1, cat2, dcat2, 2},
                       {"down1", "enc1b", "enc1a", p.down1, p.enc1a, p.down0, cat1, dcat1, 1},
                       {"down0", "enc0b", "enc0a", p.down0, p.enc0a, p.x, cat0, dcat0, 0}};
  for (const Enc& en : encs) {
    const int l = en.l;
    const int C = c0 << l;      // channels of level l
    const int Cd = 2 * C;       // channels of the down output
    const Layer& Ld = layer(c, en.down);
    BWD(prep(c, P[l + 1], Cd, Ld.np, gB, Cd, nullptr, 0, A(en.act_down), Cd, gpre));
    BWD(conv_wgrad(c, p, Ld, View{en.cat + C, C, 2 * C}, B, Nl[l], Nl[l + 1], CM_DOWN3, 1, gpre));
    BWD(conv_dgrad(c, Ld, gpre, B, Nl[l + 1], gA));  // fine grid [P_l][C]
    // enc_b output = skip: gradient from the down path plus the concat slice
    const Layer& Lb = layer(c, en.b);
    BWD(prep(c, P[l], C, Lb.np, gA, C, en.dcat + C, 2 * C, en.cat + C, 2 * C, gpre));
    BWD(conv_wgrad(c, p, Lb, View{A(en.act_a), C, C}, B, Nl[l], Nl[l], CM_CONV3, 1, gpre));
    BWD(conv_dgrad(c, Lb, gpre, B, Nl[l], gB));
    const Layer& La = layer(c, en.a);
    BWD(prep(c, P[l], C, La.np, gB, C, nullptr, 0, A(en.act_a), C, gpre));
    const int cin_a = l == 0 ? 8 : C;
    BWD(conv_wgrad(c, p, La, View{A(en.in_a), cin_a, cin_a}, B, Nl[l], Nl[l], CM_CONV3, 1, gpre));
    if (l > 0) BWD(conv_dgrad(c, La, gpre, B, Nl[l], gB));  // gradient of down_{l-1} output
  }
#undef BWD
  return hipSuccess;
}

lshom_status check_ws(lshom_cnn* c, int B, int N, bool training) {
  if (!c->params_set) return fail(c, LSHOM_ERR_STATE, "parameters not set");
  if (!c->ws) return fail(c, LSHOM_ERR_WORKSPACE, "no workspace");
  if (B != c->ws_B || N != c->ws_N) return fail(c, LSHOM_ERR_WORKSPACE, "workspace set for another (batch, n)");
  if (training && !c->ws_train) return fail(c, LSHOM_ERR_WORKSPACE, "workspace has no training buffers");
  return LSHOM_OK;
}

// Grids of one layer call on the workspace shape (batch B, side N): the
// output side Ho, the input side Hi, the convolution mode and the
// upsampling factor of the input read.
struct LayerGeom {
  int Hi, Ho, mode, up;
};

LayerGeom layer_geom(const lshom_cnn* c, int li, int N) {
  static const int lev_out[] = {0, 0, 1, 1, 1, 2, 2, 2, 3, 3, 3, 2, 2, 2, 1, 1, 1, 0, 0, 0, 0};
  const Layer& L = c->layers[li];
  int Ho = N;
  for (int l = 0; l < lev_out[li]; ++l) Ho /= 3;
  LayerGeom g{Ho, Ho, CM_CONV3, 1};
  if (L.kind == K_DOWN3) {
    g.Hi = 3 * Ho;
    g.mode = CM_DOWN3;
  } else if (L.kind == K_CONV1) {
    g.mode = CM_POINT;
  } else if (L.name.compare(0, 2, "up") == 0) {
    g.Hi = Ho / 3;
    g.up = 3;
  }
  return g;
}

bool shape_ok(int B, int N) { return B >= 1 && N >= 27 && N % 27 == 0 && (long long)B * N * N < (1LL << 31) / 64; }

}  // namespace

extern "C" {

lshom_status lshom_cnn_create(lshom_cnn** out, int device, void* hip_stream, int base_channels) {
  if (!out) return LSHOM_ERR_INVALID_ARG;
  *out = nullptr;
  if (base_channels < 8 || base_channels % 8 != 0 || base_channels > 64) return LSHOM_ERR_INVALID_ARG;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return LSHOM_ERR_HIP;
  lshom_cnn* c = new lshom_cnn();
  c->device = device;
  c->c0 = base_channels;
  c->user_stream = static_cast<hipStream_t>(hip_stream);
  DeviceGuard g(device);
  if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev, hipEventDisableTiming) != hipSuccess) {
    if (c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return LSHOM_ERR_HIP;
  }
  build_layers(c);
  *out = c;
  return LSHOM_OK;
}

void lshom_cnn_destroy(lshom_cnn* c) {
  if (!c) return;
  DeviceGuard g(c->device);
  (void)hipStreamSynchronize(c->stream);
  if (c->ev) (void)hipEventDestroy(c->ev);
  if (c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

const char* lshom_cnn_last_error(const lshom_cnn* c) { return c ? c->err.c_str() : "null network"; }

lshom_status lshom_cnn_param_size(lshom_cnn* c, int64_t* n_params, size_t* buffer_bytes) {
  if (!c) return LSHOM_ERR_INVALID_ARG;
  if (n_params) *n_params = c->n_compact;
  if (buffer_bytes) *buffer_bytes = c->n_el * (4 * sizeof(float) + 2 * sizeof(bf16_t)) + 256;
  return LSHOM_OK;
}

lshom_status lshom_cnn_set_param_buffer(lshom_cnn* c, void* dev, size_t bytes) {
  if (!c) return LSHOM_ERR_INVALID_ARG;
  size_t need = 0;
  lshom_cnn_param_size(c, nullptr, &need);
  if (!dev || bytes < need || (reinterpret_cast<uintptr_t>(dev) & 255))
    return fail(c, LSHOM_ERR_WORKSPACE, "parameter buffer NULL, unaligned or too small");
  c->pbuf = static_cast<char*>(dev);
  c->pbytes = bytes;
  char* q = c->pbuf;
  c->w = reinterpret_cast<float*>(q);
  q += c->n_el * 4;
  c->g = reinterpret_cast<float*>(q);
  q += c->n_el * 4;
  c->m = reinterpret_cast<float*>(q);
  q += c->n_el * 4;
  c->v = reinterpret_cast<float*>(q);
  q += c->n_el * 4;
  c->w16 = reinterpret_cast<bf16_t*>(q);
  q += c->n_el * 2;
  c->wt16 = reinterpret_cast<bf16_t*>(q);
  c->params_set = false;
  return LSHOM_OK;
}

lshom_status lshom_cnn_set_params(lshom_cnn* c, const float* host, int64_t n) {
  if (!c || !host) return LSHOM_ERR_INVALID_ARG;
  if (!c->pbuf) return fail(c, LSHOM_ERR_STATE, "parameter buffer not set");
  if (n != c->n_compact) return fail(c, LSHOM_ERR_INVALID_ARG, "parameter count mismatch");
  std::vector<float> padded(c->n_el, 0.f);
  long long k = 0;
  for (const Layer& L : c->layers) {
    for (int t = 0; t < L.taps; ++t)
      for (int ci = 0; ci < L.cin_real; ++ci)
        for (int o = 0; o < L.cout; ++o) padded[L.w_off + ((size_t)t * L.cin + ci) * L.np + o] = host[k++];
    for (int o = 0; o < L.cout; ++o) padded[L.b_off + o] = host[k++];
  }
  DeviceGuard g(c->device);
  CNN_TRY(c, order_after_user(c));
  CNN_TRY(c, hipMemcpyAsync(c->w, padded.data(), c->n_el * 4, hipMemcpyHostToDevice, c->stream));
  CNN_TRY(c, launch_fill_f32(c->g, (long long)c->n_el, 0.f, c->stream));
  CNN_TRY(c, launch_fill_f32(c->m, (long long)c->n_el, 0.f, c->stream));
  CNN_TRY(c, launch_fill_f32(c->v, (long long)c->n_el, 0.f, c->stream));
  // the gaps between the layers' bfloat16 copies are never written: clear both copies once
  CNN_TRY(c, launch_fill_f32(reinterpret_cast<float*>(c->w16), (long long)c->n_el, 0.f, c->stream));
  CNN_TRY(c, cast_all(c));
  CNN_TRY(c, hipStreamSynchronize(c->stream));
  c->adam_t = 0;
  c->params_set = true;
  return LSHOM_OK;
}

static lshom_status get_compact(lshom_cnn* c, const float* dev, float* host, int64_t n) {
  if (!c || !host) return LSHOM_ERR_INVALID_ARG;
  if (!c->params_set) return fail(c, LSHOM_ERR_STATE, "parameters not set");
  if (n != c->n_compact) return fail(c, LSHOM_ERR_INVALID_ARG, "parameter count mismatch");
  std::vector<float> padded(c->n_el);
  DeviceGuard g(c->device);
  CNN_TRY(c, order_after_user(c));
  CNN_TRY(c, hipMemcpyAsync(padded.data(), dev, c->n_el * 4, hipMemcpyDeviceToHost, c->stream));
  CNN_TRY(c, hipStreamSynchronize(c->stream));
  long long k = 0;
  for (const Layer& L : c->layers) {
    for (int t = 0; t < L.taps; ++t)
      for (int ci = 0; ci < L.cin_real; ++ci)
        for (int o = 0; o < L.cout; ++o) host[k++] = padded[L.w_off + ((size_t)t * L.cin + ci) * L.np + o];
    for (int o = 0; o < L.cout; ++o) host[k++] = padded[L.b_off + o];
  }
  return LSHOM_OK;
}

lshom_status lshom_cnn_get_params(lshom_cnn* c, float* host, int64_t n) { return get_compact(c, c ? c->w : nullptr, host, n); }
lshom_status lshom_cnn_get_grads(lshom_cnn* c, float* host, int64_t n) { return get_compact(c, c ? c->g : nullptr, host, n); }

lshom_status lshom_cnn_workspace_size(lshom_cnn* c, int batch, int n, int training, size_t* bytes) {
  if (!c || !bytes) return LSHOM_ERR_INVALID_ARG;
  if (!shape_ok(batch, n)) return fail(c, LSHOM_ERR_INVALID_ARG, "batch >= 1 and n a multiple of 27 required");
  *bytes = make_plan(c, batch, n, training).total + 256;
  return LSHOM_OK;
}

lshom_status lshom_cnn_set_workspace(lshom_cnn* c, void* dev, size_t bytes, int batch, int n, int training) {
  if (!c) return LSHOM_ERR_INVALID_ARG;
  size_t need = 0;
  lshom_status s = lshom_cnn_workspace_size(c, batch, n, training, &need);
  if (s != LSHOM_OK) return s;
  if (!dev || bytes < need - 256 || (reinterpret_cast<uintptr_t>(dev) & 255))
    return fail(c, LSHOM_ERR_WORKSPACE, "workspace NULL, unaligned or too small");
  c->ws = static_cast<char*>(dev);
  c->ws_bytes = bytes;
  c->ws_B = batch;
  c->ws_N = n;
  c->ws_train = training ? 1 : 0;
  return LSHOM_OK;
}

lshom_status lshom_cnn_forward(lshom_cnn* c, const uint8_t* phase_dev, const float* log10_rho_dev, int batch, int n,
                               int load_axis, int scale, double* e_dev, float* raw_dev) {
  if (!c || !phase_dev || !log10_rho_dev) return LSHOM_ERR_INVALID_ARG;
  if (load_axis != 0 && load_axis != 1) return fail(c, LSHOM_ERR_INVALID_ARG, "load_axis must be 0 or 1");
  if ((scale != 1 && scale != 3) || n % scale != 0) return fail(c, LSHOM_ERR_INVALID_ARG, "scale must be 1 or 3 and divide n");
  const int nc = n / scale;
  lshom_status s = check_ws(c, batch, nc, false);
  if (s != LSHOM_OK) return s;
  const Plan p = make_plan(c, batch, nc, c->ws_train);
  DeviceGuard g(c->device);
  CNN_TRY(c, order_after_user(c));
  CNN_TRY(c, forward(c, p, batch, phase_dev, log10_rho_dev, load_axis, scale));
  const float* out = at<float>(c, p.out);
  if (e_dev) CNN_TRY(c, launch_make_field(batch, nc, out, load_axis, scale, e_dev, c->stream));
  if (raw_dev)
    CNN_TRY(c, hipMemcpyAsync(raw_dev, out, (size_t)batch * nc * nc * 2 * sizeof(float), hipMemcpyDeviceToDevice,
                              c->stream));
  CNN_TRY(c, hipStreamSynchronize(c->stream));
  c->err.clear();
  return LSHOM_OK;
}

lshom_status lshom_cnn_train_step(lshom_cnn* c, const uint8_t* phase_dev, const float* log10_rho_dev,
                                  const double* e_dev, int batch, int n, float lr, int update, double* loss_host) {
  if (!c || !phase_dev || !log10_rho_dev || !e_dev) return LSHOM_ERR_INVALID_ARG;
  if (!(lr >= 0.f)) return fail(c, LSHOM_ERR_INVALID_ARG, "lr must be >= 0");
  lshom_status s = check_ws(c, batch, n, true);
  if (s != LSHOM_OK) return s;
  const Plan p = make_plan(c, batch, n, 1);
  DeviceGuard g(c->device);
  CNN_TRY(c, order_after_user(c));
  CNN_TRY(c, forward(c, p, batch, phase_dev, log10_rho_dev, 0, 1));
  double* part = at<double>(c, p.part);
  double* loss = at<double>(c, p.loss);
  CNN_TRY(c, launch_rel_mse(batch, n, at<float>(c, p.out), e_dev, part, loss, at<float>(c, p.gout), c->stream));
  CNN_TRY(c, backward(c, p, batch));
  if (update) {
    c->adam_t += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - std::pow(b1, (float)c->adam_t);
    const float c2 = 1.f - std::pow(b2, (float)c->adam_t);
    CNN_TRY(c, launch_adam((long long)c->n_el, c->w, c->g, c->m, c->v, lr, b1, b2, 1e-8f, c1, c2, c->stream));
    CNN_TRY(c, cast_all(c));
  }
  double h = 0.0;
  CNN_TRY(c, hipMemcpyAsync(&h, loss, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  CNN_TRY(c, hipStreamSynchronize(c->stream));
  if (loss_host) *loss_host = h;
  c->err.clear();
  return LSHOM_OK;
}

lshom_status lshom_cnn_layer_forward(lshom_cnn* c, int layer, const uint16_t* x_dev, uint16_t* y_dev,
                                     float* yf_dev) {
  if (!c || !x_dev || (!y_dev && !yf_dev)) return LSHOM_ERR_INVALID_ARG;
  if (layer < 0 || layer >= (int)c->layers.size()) return fail(c, LSHOM_ERR_INVALID_ARG, "layer index out of range");
  lshom_status s = check_ws(c, c->ws_B, c->ws_N, false);
  if (s != LSHOM_OK) return s;
  const Layer& L = c->layers[layer];
  const LayerGeom gm = layer_geom(c, layer, c->ws_N);
  DeviceGuard g(c->device);
  CNN_TRY(c, order_after_user(c));
  CNN_TRY(c, conv_fwd(c, L, View{x_dev, L.cin, L.cin}, c->ws_B, gm.Hi, gm.Ho, gm.mode, gm.up, y_dev, L.cout, yf_dev,
                      L.cout, L.kind != K_CONV1));
  CNN_TRY(c, hipStreamSynchronize(c->stream));
  c->err.clear();
  return LSHOM_OK;
}

lshom_status lshom_cnn_layer_dgrad(lshom_cnn* c, int layer, const uint16_t* gy_dev, float* gx_dev) {
  if (!c || !gy_dev || !gx_dev) return LSHOM_ERR_INVALID_ARG;
  if (layer < 0 || layer >= (int)c->layers.size()) return fail(c, LSHOM_ERR_INVALID_ARG, "layer index out of range");
  lshom_status s = check_ws(c, c->ws_B, c->ws_N, true);
  if (s != LSHOM_OK) return s;
  const Layer& L = c->layers[layer];
  const LayerGeom gm = layer_geom(c, layer, c->ws_N);
  const Plan p = make_plan(c, c->ws_B, c->ws_N, 1);
  DeviceGuard g(c->device);
  CNN_TRY(c, order_after_user(c));
  if (gm.up == 3) {
    // the gradient of the upsampled input on the fine grid, then the adjoint
    // of the upsampling (sum over each 3 x 3 block)
    float* fine = at<float>(c, p.gA);
    CNN_TRY(c, conv_dgrad(c, L, gy_dev, c->ws_B, gm.Ho, fine));
    CNN_TRY(c, launch_pool3_sum(c->ws_B, gm.Hi, gm.Hi, L.cin, fine, gx_dev, c->stream));
  } else {
    CNN_TRY(c, conv_dgrad(c, L, gy_dev, c->ws_B, gm.Ho, gx_dev));
  }
  CNN_TRY(c, hipStreamSynchronize(c->stream));
  c->err.clear();
  return LSHOM_OK;
}

lshom_status lshom_cnn_layer_wgrad(lshom_cnn* c, int layer, const uint16_t* x_dev, const uint16_t* gy_dev) {
  if (!c || !x_dev || !gy_dev) return LSHOM_ERR_INVALID_ARG;
  if (layer < 0 || layer >= (int)c->layers.size()) return fail(c, LSHOM_ERR_INVALID_ARG, "layer index out of range");
  lshom_status s = check_ws(c, c->ws_B, c->ws_N, true);
  if (s != LSHOM_OK) return s;
  const Layer& L = c->layers[layer];
  const LayerGeom gm = layer_geom(c, layer, c->ws_N);
  const Plan p = make_plan(c, c->ws_B, c->ws_N, 1);
  DeviceGuard g(c->device);
  CNN_TRY(c, order_after_user(c));
  CNN_TRY(c, conv_wgrad(c, p, L, View{x_dev, L.cin, L.cin}, c->ws_B, gm.Hi, gm.Ho, gm.mode, gm.up, gy_dev));
  CNN_TRY(c, hipStreamSynchronize(c->stream));
  c->err.clear();
  return LSHOM_OK;
}

}  // extern "C"
