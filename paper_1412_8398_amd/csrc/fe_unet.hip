// C ABI of the warm-start U-Net (include/fe_nn.h): parameters, workspace,
// forward, backward and Adam, every step in the library's kernels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/fe_nn.h"
#include "fe_error.h"
#include "fe_nn.h"

using namespace fe;
using namespace fe::nn;

namespace {

struct LayerDef {
  int cin, cout;
};

// enc1a enc1b enc2a enc2b enc3a enc3b bota botb dec3a dec3b dec2a dec2b dec1a dec1b
constexpr int kLayers = 14;
const LayerDef kDef[kLayers] = {{8, 16},  {16, 16},   {16, 32},  {32, 32}, {32, 64},  {64, 64},  {64, 128},
                                {128, 128}, {192, 64}, {64, 64}, {96, 32}, {32, 32}, {48, 16}, {16, 16}};
enum { ENC1A, ENC1B, ENC2A, ENC2B, ENC3A, ENC3B, BOTA, BOTB, DEC3A, DEC3B, DEC2A, DEC2B, DEC1A, DEC1B };

long long param_count() {
  long long n = 0;
  for (const auto& l : kDef) n += 27LL * l.cin * l.cout + l.cout;
  return n + 16 * 6 + 6;
}

// SplitMix64 and Box-Muller for the initial weights
struct SplitMix64 {
  uint64_t s;
  uint64_t next() {
    s += 0x9E3779B97F4A7C15ull;
    uint64_t z = s;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  double uniform() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }
  double normal() {
    const double u1 = 1.0 - uniform(), u2 = uniform();  // u1 in (0, 1]
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(2.0 * M_PI * u2);
  }
};

template <typename T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
  hipError_t ensure(size_t count) {
    if (count <= n) return hipSuccess;
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
    hipError_t e = hipMalloc((void**)&p, count * sizeof(T));
    if (e == hipSuccess) n = count;
    return e;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
};

Grid3 coarse(const Grid3& g) { return Grid3{g.nx / 2, g.ny / 2, g.nz / 2, g.nb}; }

}  // namespace

struct fe_unet {
  fe_unet_config cfg;
  hipStream_t s = nullptr;
  long long nparam = 0;
  long long off_w[kLayers], off_b[kLayers], off_hw = 0, off_hb = 0;
  float *theta = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
  int t = 0;
  uint16_t* wf[kLayers] = {};  // packed forward weights
  uint16_t* wb[kLayers] = {};  // packed input-gradient weights
  bool packed = false;
  // workspace
  Grid3 shape{0, 0, 0, 0};
  bool have_grads = false;
  DevBuf<uint16_t> act, gbuf;
  DevBuf<float> wpart, bpart;
  DevBuf<double> hpart, sums, loss;
  DevBuf<FeatTab> tabs;
  // activation pointers
  uint16_t *x0, *e1a, *e1, *p1, *e2a, *e2, *p2, *e3a, *e3, *p3, *ba, *bt, *cat3, *d3a, *d3, *cat2, *d2a, *d2, *cat1,
      *d1a, *d1;
  // gradient pointers
  uint16_t *gd1, *gd1a, *gcat1, *gd2, *gd2a, *gcat2, *gd3, *gd3a, *gcat3, *gbt, *gba, *gp3, *ge3, *ge3a, *gp2, *ge2,
      *ge2a, *gp1, *ge1, *ge1a;
};

static void free_net(fe_unet* n) {
  void* b[] = {n->theta, n->grad, n->m, n->v};
  for (void* x : b)
    if (x) (void)hipFree(x);
  for (int l = 0; l < kLayers; ++l) {
    if (n->wf[l]) (void)hipFree(n->wf[l]);
    if (n->wb[l]) (void)hipFree(n->wb[l]);
  }
  n->act.release();
  n->gbuf.release();
  n->wpart.release();
  n->bpart.release();
  n->hpart.release();
  n->sums.release();
  n->loss.release();
  n->tabs.release();
  delete n;
}

static fe_status repack(fe_unet* n) {
  for (int l = 0; l < kLayers; ++l) {
    pack_weights(n->theta + n->off_w[l], kDef[l].cin, kDef[l].cout, 0, n->wf[l], n->s);
    if (n->wb[l]) pack_weights(n->theta + n->off_w[l], kDef[l].cin, kDef[l].cout, 1, n->wb[l], n->s);
  }
  HIP_TRY(hipGetLastError());
  n->packed = true;
  return FE_OK;
}

extern "C" void fe_unet_config_default(fe_unet_config* c) {
  if (!c) return;
  std::memset(c, 0, sizeof *c);
  c->struct_size = sizeof(fe_unet_config);
  c->seed = 1412839801ull;
  c->lr = 1e-3f;
  c->beta1 = 0.9f;
  c->beta2 = 0.999f;
  c->adam_eps = 1e-8f;
  c->hip_stream = nullptr;
}

extern "C" int64_t fe_unet_param_count(void) { return param_count(); }

extern "C" fe_status fe_unet_create(const fe_unet_config* cfg, fe_unet** out) {
  if (!out) return fail(FE_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  fe_unet_config c;
  fe_unet_config_default(&c);
  if (cfg) {
    if (cfg->struct_size != sizeof(fe_unet_config))
      return fail(FE_ERR_INVALID_ARG, "fe_unet_config.struct_size is %u, expected %zu", cfg->struct_size,
                  sizeof(fe_unet_config));
    c = *cfg;
  }
  if (!(c.lr > 0.f) || !(c.beta1 >= 0.f && c.beta1 < 1.f) || !(c.beta2 >= 0.f && c.beta2 < 1.f) || !(c.adam_eps > 0.f))
    return fail(FE_ERR_INVALID_ARG, "Adam settings out of range");
  fe_unet* n = new fe_unet();
  n->cfg = c;
  n->s = (hipStream_t)c.hip_stream;
  long long o = 0;
  for (int l = 0; l < kLayers; ++l) {
    n->off_w[l] = o;
    o += 27LL * kDef[l].cin * kDef[l].cout;
    n->off_b[l] = o;
    o += kDef[l].cout;
  }
  n->off_hw = o;
  o += 96;
  n->off_hb = o;
  o += 6;
  n->nparam = o;
  std::vector<float> h((size_t)o, 0.f);
  SplitMix64 rng{c.seed};
  for (int l = 0; l < kLayers; ++l) {
    const double sd = std::sqrt(2.0 / (27.0 * kDef[l].cin));
    for (long long i = 0; i < 27LL * kDef[l].cin * kDef[l].cout; ++i) h[n->off_w[l] + i] = (float)(sd * rng.normal());
  }
  for (int i = 0; i < 96; ++i) h[n->off_hw + i] = (float)(std::sqrt(2.0 / 16.0) * rng.normal());
  hipError_t e = hipSuccess;
  auto al = [&](void** p, size_t bytes) {
    if (e == hipSuccess) e = hipMalloc(p, bytes);
  };
  al((void**)&n->theta, o * sizeof(float));
  al((void**)&n->grad, o * sizeof(float));
  al((void**)&n->m, o * sizeof(float));
  al((void**)&n->v, o * sizeof(float));
  for (int l = 0; l < kLayers; ++l) {
    al((void**)&n->wf[l], packed_elems(kDef[l].cin, kDef[l].cout) * sizeof(uint16_t));
    if (l != ENC1A) al((void**)&n->wb[l], packed_elems(kDef[l].cout, kDef[l].cin) * sizeof(uint16_t));
  }
  if (e != hipSuccess) {
    free_net(n);
    return fail(e == hipErrorOutOfMemory ? FE_ERR_OOM : FE_ERR_DEVICE, "parameters: %s", hipGetErrorString(e));
  }
  if ((e = hipMemcpy(n->theta, h.data(), o * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemset(n->grad, 0, o * sizeof(float))) != hipSuccess ||
      (e = hipMemset(n->m, 0, o * sizeof(float))) != hipSuccess ||
      (e = hipMemset(n->v, 0, o * sizeof(float))) != hipSuccess) {
    free_net(n);
    return fail(FE_ERR_DEVICE, "parameters: %s", hipGetErrorString(e));
  }
  fe_status st = repack(n);
  if (st != FE_OK) {
    free_net(n);
    return st;
  }
  *out = n;
  return FE_OK;
}

extern "C" void fe_unet_destroy(fe_unet* n) {
  if (!n) return;
  (void)hipStreamSynchronize(n->s);
  free_net(n);
}

extern "C" fe_status fe_unet_set_learning_rate(fe_unet* n, float lr) {
  if (!n) return fail(FE_ERR_INVALID_ARG, "net is NULL");
  if (!(lr > 0.f) || !std::isfinite(lr)) return fail(FE_ERR_INVALID_ARG, "learning rate must be finite and > 0");
  n->cfg.lr = lr;
  return FE_OK;
}

extern "C" fe_status fe_unet_get_params(fe_unet* n, float* h) {
  if (!n || !h) return fail(FE_ERR_INVALID_ARG, "net or buffer is NULL");
  HIP_TRY(hipMemcpyAsync(h, n->theta, n->nparam * sizeof(float), hipMemcpyDeviceToHost, n->s));
  HIP_TRY(hipStreamSynchronize(n->s));
  return FE_OK;
}

extern "C" fe_status fe_unet_get_grads(fe_unet* n, float* h) {
  if (!n || !h) return fail(FE_ERR_INVALID_ARG, "net or buffer is NULL");
  HIP_TRY(hipMemcpyAsync(h, n->grad, n->nparam * sizeof(float), hipMemcpyDeviceToHost, n->s));
  HIP_TRY(hipStreamSynchronize(n->s));
  return FE_OK;
}

extern "C" fe_status fe_unet_set_params(fe_unet* n, const float* h) {
  if (!n || !h) return fail(FE_ERR_INVALID_ARG, "net or buffer is NULL");
  for (long long i = 0; i < n->nparam; ++i)
    if (!std::isfinite(h[i])) return fail(FE_ERR_INVALID_ARG, "parameter %lld is not finite", i);
  HIP_TRY(hipMemcpyAsync(n->theta, h, n->nparam * sizeof(float), hipMemcpyHostToDevice, n->s));
  HIP_TRY(hipMemsetAsync(n->m, 0, n->nparam * sizeof(float), n->s));
  HIP_TRY(hipMemsetAsync(n->v, 0, n->nparam * sizeof(float), n->s));
  n->t = 0;
  fe_status st = repack(n);
  if (st != FE_OK) return st;
  HIP_TRY(hipStreamSynchronize(n->s));
  return FE_OK;
}

// ---------------------------------------------------------------------------
// workspace
// ---------------------------------------------------------------------------
static fe_status ensure_workspace(fe_unet* n, const Grid3& g, bool grads) {
  const long long V1 = g.voxels(), V2 = V1 / 8, V3 = V1 / 64, V4 = V1 / 512;
  // activation channels per level; the concatenated decoder inputs only for
  // training (inference reads them in place)
  const long long cat_elems = grads ? V1 * 48 + V2 * 96 + V3 * 192 : 0;
  const long long act_elems = V1 * (8 + 16 + 16 + 16 + 16) + V2 * (16 + 32 + 32 + 32 + 32) +
                              V3 * (32 + 64 + 64 + 64 + 64) + V4 * (64 + 128 + 128) + cat_elems;
  const long long grad_elems = V1 * (16 + 16 + 48 + 16 + 16) + V2 * (32 + 32 + 96 + 32 + 32 + 16) +
                               V3 * (64 + 64 + 192 + 64 + 64 + 32) + V4 * (128 + 128 + 64);
  HIP_TRY(n->act.ensure((size_t)act_elems));
  uint16_t* a = n->act.p;
  auto take = [&](long long cnt) {
    uint16_t* r = a;
    a += cnt;
    return r;
  };
  n->x0 = take(V1 * 8);
  n->e1a = take(V1 * 16);
  n->e1 = take(V1 * 16);
  n->cat1 = grads ? take(V1 * 48) : nullptr;
  n->d1a = take(V1 * 16);
  n->d1 = take(V1 * 16);
  n->p1 = take(V2 * 16);
  n->e2a = take(V2 * 32);
  n->e2 = take(V2 * 32);
  n->cat2 = grads ? take(V2 * 96) : nullptr;
  n->d2a = take(V2 * 32);
  n->d2 = take(V2 * 32);
  n->p2 = take(V3 * 32);
  n->e3a = take(V3 * 64);
  n->e3 = take(V3 * 64);
  n->cat3 = grads ? take(V3 * 192) : nullptr;
  n->d3a = take(V3 * 64);
  n->d3 = take(V3 * 64);
  n->p3 = take(V4 * 64);
  n->ba = take(V4 * 128);
  n->bt = take(V4 * 128);
  HIP_TRY(n->tabs.ensure((size_t)g.nb));
  HIP_TRY(n->hpart.ensure((size_t)g.nb * head_blocks(g) * 103 + 64));
  HIP_TRY(n->sums.ensure((size_t)g.nb * 12));
  HIP_TRY(n->loss.ensure(1));
  if (grads) {
    HIP_TRY(n->gbuf.ensure((size_t)grad_elems));
    uint16_t* q = n->gbuf.p;
    auto tg = [&](long long cnt) {
      uint16_t* r = q;
      q += cnt;
      return r;
    };
    n->gd1 = tg(V1 * 16);
    n->gd1a = tg(V1 * 16);
    n->gcat1 = tg(V1 * 48);
    n->ge1 = tg(V1 * 16);
    n->ge1a = tg(V1 * 16);
    n->gd2 = tg(V2 * 32);
    n->gd2a = tg(V2 * 32);
    n->gcat2 = tg(V2 * 96);
    n->ge2 = tg(V2 * 32);
    n->ge2a = tg(V2 * 32);
    n->gp1 = tg(V2 * 16);
    n->gd3 = tg(V3 * 64);
    n->gd3a = tg(V3 * 64);
    n->gcat3 = tg(V3 * 192);
    n->ge3 = tg(V3 * 64);
    n->ge3a = tg(V3 * 64);
    n->gp2 = tg(V3 * 32);
    n->gbt = tg(V4 * 128);
    n->gba = tg(V4 * 128);
    n->gp3 = tg(V4 * 64);
    size_t wp = 0;
    Grid3 lg[kLayers] = {g, g, coarse(g), coarse(g), coarse(coarse(g)), coarse(coarse(g)),
                         coarse(coarse(coarse(g))), coarse(coarse(coarse(g))), coarse(coarse(g)), coarse(coarse(g)),
                         coarse(g), coarse(g), g, g};
    for (int l = 0; l < kLayers; ++l) {
      const size_t f = conv3_wgrad_partial_floats(kDef[l].cin, kDef[l].cout, lg[l]);
      if (f > wp) wp = f;
    }
    HIP_TRY(n->wpart.ensure(wp));
    HIP_TRY(n->bpart.ensure(512 * 128));
  }
  n->shape = g;
  return FE_OK;
}

static fe_status validate_batch(const fe_unet_batch* b, Grid3* g) {
  if (!b) return fail(FE_ERR_INVALID_ARG, "batch is NULL");
  if (b->batch < 1 || b->batch > 65535) return fail(FE_ERR_INVALID_ARG, "batch must be in [1, 65535]");
  const int n[3] = {b->grid.nx, b->grid.ny, b->grid.nz};
  for (int a = 0; a < 3; ++a)
    if (n[a] < 8 || n[a] % 8 != 0 || n[a] > 2048)
      return fail(FE_ERR_UNSUPPORTED, "grid dimension %d = %d: the network needs multiples of 8 in [8, 2048]", a, n[a]);
  if (!b->phase || !b->materials || !b->macro_strain) return fail(FE_ERR_INVALID_ARG, "batch arrays are NULL");
  for (int s = 0; s < b->batch; ++s) {
    const fe_materials& m = b->materials[s];
    if (m.n_phases < 1 || m.n_phases > 256 || !m.E || !m.nu)
      return fail(FE_ERR_INVALID_ARG, "sample %d: n_phases must be in [1, 256] with E and nu set", s);
    for (int p = 0; p < m.n_phases; ++p)
      if (!(std::isfinite(m.E[p]) && m.E[p] > 0.0 && std::isfinite(m.nu[p]) && m.nu[p] > -1.0 && m.nu[p] < 0.5))
        return fail(FE_ERR_INVALID_ARG, "sample %d phase %d: need E > 0 and -1 < nu < 0.5", s, p);
    for (int q = 0; q < 6; ++q)
      if (!std::isfinite(b->macro_strain[6 * s + q])) return fail(FE_ERR_INVALID_ARG, "sample %d: macro strain", s);
  }
  *g = Grid3{b->grid.nx, b->grid.ny, b->grid.nz, b->batch};
  return FE_OK;
}

static fe_status upload_tabs(fe_unet* n, const fe_unet_batch* b) {
  std::vector<FeatTab> t((size_t)b->batch);
  for (int s = 0; s < b->batch; ++s) {
    FeatTab& f = t[s];
    std::memset(&f, 0, sizeof f);
    const fe_materials& m = b->materials[s];
    for (int p = 0; p < m.n_phases; ++p) {
      f.logE[p] = (float)(std::log10(m.E[p]) / 3.0);
      f.nu[p] = (float)(10.0 * (m.nu[p] - 0.3));
    }
    for (int q = 0; q < 6; ++q) f.macro[q] = (float)b->macro_strain[6 * s + q];
  }
  HIP_TRY(hipMemcpyAsync(n->tabs.p, t.data(), t.size() * sizeof(FeatTab), hipMemcpyHostToDevice, n->s));
  HIP_TRY(hipStreamSynchronize(n->s));  // t is pageable and goes out of scope
  return FE_OK;
}

// ---------------------------------------------------------------------------
// forward / backward
// ---------------------------------------------------------------------------
static void conv(fe_unet* n, int l, const uint16_t* x, uint16_t* y, const Grid3& g) {
  conv3_forward(kDef[l].cin, kDef[l].cout, x, nullptr, n->wf[l], n->theta + n->off_b[l], 1, y, g, n->s);
}

// decoder layer l on [up2(coarse), skip] read in place (no concatenated input)
static void conv_cat(fe_unet* n, int l, int ca, const uint16_t* coarse, const uint16_t* skip, uint16_t* y,
                     const Grid3& g) {
  conv3_forward_cat(kDef[l].cin, kDef[l].cout, ca, coarse, skip, n->wf[l], n->theta + n->off_b[l], 1, y, g, n->s);
}

// With cat_in_place the decoder layers read their concatenated inputs in place
// (inference); training keeps the concatenations, which the weight gradients read.
static void forward(fe_unet* n, const uint8_t* phase, const Grid3& g1, bool cat_in_place) {
  const Grid3 g2 = coarse(g1), g3 = coarse(g2), g4 = coarse(g3);
  features(phase, n->tabs.p, n->x0, g1, n->s);
  conv(n, ENC1A, n->x0, n->e1a, g1);
  conv(n, ENC1B, n->e1a, n->e1, g1);
  pool2(n->e1, 16, n->p1, g1, n->s);
  conv(n, ENC2A, n->p1, n->e2a, g2);
  conv(n, ENC2B, n->e2a, n->e2, g2);
  pool2(n->e2, 32, n->p2, g2, n->s);
  conv(n, ENC3A, n->p2, n->e3a, g3);
  conv(n, ENC3B, n->e3a, n->e3, g3);
  pool2(n->e3, 64, n->p3, g3, n->s);
  conv(n, BOTA, n->p3, n->ba, g4);
  conv(n, BOTB, n->ba, n->bt, g4);
  if (cat_in_place) {
    conv_cat(n, DEC3A, 128, n->bt, n->e3, n->d3a, g3);
  } else {
    up_concat(n->bt, 128, n->e3, 64, n->cat3, g3, n->s);
    conv(n, DEC3A, n->cat3, n->d3a, g3);
  }
  conv(n, DEC3B, n->d3a, n->d3, g3);
  if (cat_in_place) {
    conv_cat(n, DEC2A, 64, n->d3, n->e2, n->d2a, g2);
  } else {
    up_concat(n->d3, 64, n->e2, 32, n->cat2, g2, n->s);
    conv(n, DEC2A, n->cat2, n->d2a, g2);
  }
  conv(n, DEC2B, n->d2a, n->d2, g2);
  if (cat_in_place) {
    conv_cat(n, DEC1A, 32, n->d2, n->e1, n->d1a, g1);
  } else {
    up_concat(n->d2, 32, n->e1, 16, n->cat1, g1, n->s);
    conv(n, DEC1A, n->cat1, n->d1a, g1);
  }
  conv(n, DEC1B, n->d1a, n->d1, g1);
}

// gradients of layer l (input x, output y after relu, upstream gradient gy of y):
// weight and bias gradients into n->grad, input gradient into gx (nullable)
static void layer_backward(fe_unet* n, int l, const uint16_t* x, const uint16_t* y, const uint16_t* gy, uint16_t* gx,
                           const Grid3& g) {
  const int ci = kDef[l].cin, co = kDef[l].cout;
  const int sets = conv3_wgrad_partials(ci, co, x, gy, y, n->wpart.p, g, n->s);
  conv3_wgrad_reduce(ci, co, n->wpart.p, sets, n->grad + n->off_w[l], n->s);
  bias_grad(gy, y, co, n->bpart.p, n->grad + n->off_b[l], g, n->s);
  if (gx) conv3_forward(co, ci, gy, y, n->wb[l], nullptr, 0, gx, g, n->s);
}

static void backward(fe_unet* n, const Grid3& g1) {
  const Grid3 g2 = coarse(g1), g3 = coarse(g2), g4 = coarse(g3);
  layer_backward(n, DEC1B, n->d1a, n->d1, n->gd1, n->gd1a, g1);
  layer_backward(n, DEC1A, n->cat1, n->d1a, n->gd1a, n->gcat1, g1);
  up_backward(n->gcat1, 32, 16, n->gd2, g1, n->s);
  layer_backward(n, DEC2B, n->d2a, n->d2, n->gd2, n->gd2a, g2);
  layer_backward(n, DEC2A, n->cat2, n->d2a, n->gd2a, n->gcat2, g2);
  up_backward(n->gcat2, 64, 32, n->gd3, g2, n->s);
  layer_backward(n, DEC3B, n->d3a, n->d3, n->gd3, n->gd3a, g3);
  layer_backward(n, DEC3A, n->cat3, n->d3a, n->gd3a, n->gcat3, g3);
  up_backward(n->gcat3, 128, 64, n->gbt, g3, n->s);
  layer_backward(n, BOTB, n->ba, n->bt, n->gbt, n->gba, g4);
  layer_backward(n, BOTA, n->p3, n->ba, n->gba, n->gp3, g4);
  pool_backward_add(n->gp3, n->gcat3, 128, 64, n->ge3, g3, n->s);
  layer_backward(n, ENC3B, n->e3a, n->e3, n->ge3, n->ge3a, g3);
  layer_backward(n, ENC3A, n->p2, n->e3a, n->ge3a, n->gp2, g3);
  pool_backward_add(n->gp2, n->gcat2, 64, 32, n->ge2, g2, n->s);
  layer_backward(n, ENC2B, n->e2a, n->e2, n->ge2, n->ge2a, g2);
  layer_backward(n, ENC2A, n->p1, n->e2a, n->ge2a, n->gp1, g2);
  pool_backward_add(n->gp1, n->gcat1, 32, 16, n->ge1, g1, n->s);
  layer_backward(n, ENC1B, n->e1a, n->e1, n->ge1, n->ge1a, g1);
  layer_backward(n, ENC1A, n->x0, n->e1a, n->ge1a, nullptr, g1);
}

extern "C" fe_status fe_unet_predict(fe_unet* n, const fe_unet_batch* b, void* out, double* seconds) {
  if (!n) return fail(FE_ERR_INVALID_ARG, "net is NULL");
  if (!out) return fail(FE_ERR_INVALID_ARG, "strain_out is NULL");
  Grid3 g;
  fe_status st = validate_batch(b, &g);
  if (st != FE_OK) return st;
  if ((st = ensure_workspace(n, g, false)) != FE_OK) return st;
  if ((st = upload_tabs(n, b)) != FE_OK) return st;
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  HIP_TRY(hipEventRecord(e0, n->s));
  forward(n, b->phase, g, true);
  head_stats(n->d1, n->theta + n->off_hw, n->theta + n->off_hb, nullptr, 0, n->hpart.p, n->sums.p, g, n->s);
  head_predict(n->d1, n->theta + n->off_hw, n->theta + n->off_hb, n->sums.p, n->tabs.p, static_cast<float*>(out), g,
               n->s);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipEventRecord(e1, n->s));
  HIP_TRY(hipEventSynchronize(e1));
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (seconds) *seconds = ms * 1e-3;
  return FE_OK;
}

static fe_status loss_grad(fe_unet* n, const fe_unet_batch* b, const void* target, int tbf16, double* loss) {
  if (!n) return fail(FE_ERR_INVALID_ARG, "net is NULL");
  if (!target) return fail(FE_ERR_INVALID_ARG, "target is NULL");
  if (tbf16 != 0 && tbf16 != 1) return fail(FE_ERR_INVALID_ARG, "target_bf16 must be 0 or 1");
  Grid3 g;
  fe_status st = validate_batch(b, &g);
  if (st != FE_OK) return st;
  if ((st = ensure_workspace(n, g, true)) != FE_OK) return st;
  if ((st = upload_tabs(n, b)) != FE_OK) return st;
  forward(n, b->phase, g, false);
  const float* hw = n->theta + n->off_hw;
  const float* hb = n->theta + n->off_hb;
  head_stats(n->d1, hw, hb, target, tbf16, n->hpart.p, n->sums.p, g, n->s);
  head_backward(n->d1, hw, hb, n->sums.p, n->tabs.p, target, tbf16, n->gd1, n->hpart.p, n->loss.p,
                n->grad + n->off_hw, n->grad + n->off_hb, g, n->s);
  backward(n, g);
  HIP_TRY(hipGetLastError());
  double l = 0.0;
  HIP_TRY(hipMemcpyAsync(&l, n->loss.p, sizeof(double), hipMemcpyDeviceToHost, n->s));
  HIP_TRY(hipStreamSynchronize(n->s));
  if (loss) *loss = l;
  if (!std::isfinite(l)) return fail(FE_DIVERGED, "loss is not finite");
  return FE_OK;
}

extern "C" fe_status fe_unet_loss_grad(fe_unet* n, const fe_unet_batch* b, const void* target, int32_t tbf16,
                                       double* loss) {
  return loss_grad(n, b, target, tbf16, loss);
}

extern "C" fe_status fe_unet_train_step(fe_unet* n, const fe_unet_batch* b, const void* target, int32_t tbf16,
                                        double* loss) {
  fe_status st = loss_grad(n, b, target, tbf16, loss);
  if (st != FE_OK) return st;
  n->t += 1;
  adam(n->theta, n->grad, n->m, n->v, n->nparam, n->cfg.lr, n->cfg.beta1, n->cfg.beta2, n->cfg.adam_eps, n->t, n->s);
  if ((st = repack(n)) != FE_OK) return st;
  HIP_TRY(hipGetLastError());
  return FE_OK;
}

// ---------------------------------------------------------------------------
// single layers
// ---------------------------------------------------------------------------
static fe_status check_shape(const fe_nn_conv_shape* s, Grid3* g) {
  if (!s) return fail(FE_ERR_INVALID_ARG, "shape is NULL");
  if (s->nx < 1 || s->ny < 1 || s->nz < 1 || s->batch < 1 || s->nx > 4096 || s->ny > 4096 || s->nz > 4096 ||
      s->batch > 65535)
    return fail(FE_ERR_INVALID_ARG, "grid or batch out of range");
  if ((long long)s->nx * s->ny * s->nz * s->batch > (1LL << 31) - 1)
    return fail(FE_ERR_UNSUPPORTED, "more than 2^31 - 1 voxels");
  *g = Grid3{s->nx, s->ny, s->nz, s->batch};
  return FE_OK;
}

static bool forward_shape(int ci, int co) {
  for (const auto& l : kDef)
    if (l.cin == ci && l.cout == co) return true;
  return false;
}

extern "C" fe_status fe_nn_conv3_forward(const fe_nn_conv_shape* sh, const uint16_t* x, const float* w, const float* b,
                                         int32_t relu, uint16_t* y, void* stream) {
  Grid3 g;
  fe_status st = check_shape(sh, &g);
  if (st != FE_OK) return st;
  if (!forward_shape(sh->c_in, sh->c_out)) return fail(FE_ERR_UNSUPPORTED, "(c_in, c_out) = (%d, %d)", sh->c_in, sh->c_out);
  if (!x || !w || !y) return fail(FE_ERR_INVALID_ARG, "x, w or y is NULL");
  hipStream_t s = (hipStream_t)stream;
  uint16_t* wp = nullptr;
  HIP_TRY(hipMalloc((void**)&wp, packed_elems(sh->c_in, sh->c_out) * sizeof(uint16_t)));
  pack_weights(w, sh->c_in, sh->c_out, 0, wp, s);
  conv3_forward(sh->c_in, sh->c_out, x, nullptr, wp, b, relu ? 1 : 0, y, g, s);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(wp);
  if (e != hipSuccess) return fail(FE_ERR_DEVICE, "conv3 forward: %s", hipGetErrorString(e));
  return FE_OK;
}

extern "C" fe_status fe_nn_conv3_forward_cat(const fe_nn_conv_shape* sh, int32_t ca, const uint16_t* coarse,
                                             const uint16_t* skip, const float* w, const float* b, int32_t relu,
                                             uint16_t* y, void* stream) {
  Grid3 g;
  fe_status st = check_shape(sh, &g);
  if (st != FE_OK) return st;
  if (!conv_cat_supported(sh->c_in, sh->c_out, ca))
    return fail(FE_ERR_UNSUPPORTED, "(c_in, c_out, c_coarse) = (%d, %d, %d)", sh->c_in, sh->c_out, ca);
  if (g.nx % 2 || g.ny % 2 || g.nz % 2) return fail(FE_ERR_INVALID_ARG, "the grid must be even in each direction");
  if (!coarse || !skip || !w || !y) return fail(FE_ERR_INVALID_ARG, "coarse, skip, w or y is NULL");
  hipStream_t s = (hipStream_t)stream;
  uint16_t* wp = nullptr;
  HIP_TRY(hipMalloc((void**)&wp, packed_elems(sh->c_in, sh->c_out) * sizeof(uint16_t)));
  pack_weights(w, sh->c_in, sh->c_out, 0, wp, s);
  conv3_forward_cat(sh->c_in, sh->c_out, ca, coarse, skip, wp, b, relu ? 1 : 0, y, g, s);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(wp);
  if (e != hipSuccess) return fail(FE_ERR_DEVICE, "conv3 forward (concatenated input): %s", hipGetErrorString(e));
  return FE_OK;
}

extern "C" fe_status fe_nn_conv3_backward_data(const fe_nn_conv_shape* sh, const uint16_t* dy, const uint16_t* ym,
                                               const float* w, uint16_t* dx, void* stream) {
  Grid3 g;
  fe_status st = check_shape(sh, &g);
  if (st != FE_OK) return st;
  if (!forward_shape(sh->c_in, sh->c_out) || sh->c_in % 16 != 0)
    return fail(FE_ERR_UNSUPPORTED, "(c_in, c_out) = (%d, %d)", sh->c_in, sh->c_out);
  if (!dy || !w || !dx) return fail(FE_ERR_INVALID_ARG, "dy, w or dx is NULL");
  hipStream_t s = (hipStream_t)stream;
  uint16_t* wp = nullptr;
  HIP_TRY(hipMalloc((void**)&wp, packed_elems(sh->c_out, sh->c_in) * sizeof(uint16_t)));
  pack_weights(w, sh->c_in, sh->c_out, 1, wp, s);
  conv3_forward(sh->c_out, sh->c_in, dy, ym, wp, nullptr, 0, dx, g, s);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(wp);
  if (e != hipSuccess) return fail(FE_ERR_DEVICE, "conv3 backward data: %s", hipGetErrorString(e));
  return FE_OK;
}

extern "C" fe_status fe_nn_conv3_backward_weight(const fe_nn_conv_shape* sh, const uint16_t* x, const uint16_t* dy,
                                                 const uint16_t* ym, float* dw, float* db, void* stream) {
  Grid3 g;
  fe_status st = check_shape(sh, &g);
  if (st != FE_OK) return st;
  if (!forward_shape(sh->c_in, sh->c_out)) return fail(FE_ERR_UNSUPPORTED, "(c_in, c_out) = (%d, %d)", sh->c_in, sh->c_out);
  if (!x || !dy || !dw) return fail(FE_ERR_INVALID_ARG, "x, dy or dw is NULL");
  hipStream_t s = (hipStream_t)stream;
  float* part = nullptr;
  HIP_TRY(hipMalloc((void**)&part, (conv3_wgrad_partial_floats(sh->c_in, sh->c_out, g) + 512 * 128) * sizeof(float)));
  const int sets = conv3_wgrad_partials(sh->c_in, sh->c_out, x, dy, ym, part, g, s);
  conv3_wgrad_reduce(sh->c_in, sh->c_out, part, sets, dw, s);
  if (db) bias_grad(dy, ym, sh->c_out, part, db, g, s);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(part);
  if (e != hipSuccess) return fail(FE_ERR_DEVICE, "conv3 backward weight: %s", hipGetErrorString(e));
  return FE_OK;
}
