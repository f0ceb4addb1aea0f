// C ABI of the solver (include/fe.h): validation, plans, the iteration loop.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <chrono>
#include <mutex>
#include <utility>
#include <string>
#include <vector>

#include "../../include/fe.h"
#include "fe_fft.h"
#include "fe_error.h"
#include "fe_kernels.h"
#include "fe_batch.h"

using namespace fe;

// ---------------------------------------------------------------------------
// host-side tables (float64)
// ---------------------------------------------------------------------------
// cos and sin of 2 pi num / den, exact at multiples of pi/2.  The angle is
// first reduced to (-pi, pi] so that small angles keep full relative accuracy
// (sin of an argument near 2 pi loses it).
static void cos_sin(long num, long den, double* c, double* s) {
  long r = ((num % den) + den) % den;  // [0, den)
  if ((4 * r) % den == 0) {
    static const double cc[4] = {1, 0, -1, 0}, ss[4] = {0, 1, 0, -1};
    int k = (int)((4 * r) / den);
    *c = cc[k];
    *s = ss[k];
    return;
  }
  if (2 * r > den) r -= den;  // (-den/2, den/2]
  const double a = 2.0 * M_PI * (double)r / (double)den;
  *c = std::cos(a);
  *s = std::sin(a);
}

// m' of eq. (12): m if 2m <= n else m - n (Nyquist at +n/2 for even n).
static long signed_mode(long m, long n) { return 2 * m <= n ? m : m - n; }

static std::vector<double> twiddles(int n) {  // exp(-2 pi i k / n), interleaved
  std::vector<double> t(2 * n);
  for (int k = 0; k < n; ++k) {
    double c, s;
    cos_sin(k, n, &c, &s);
    t[2 * k] = c;
    t[2 * k + 1] = -s;
  }
  return t;
}

static std::vector<double> wave_table(int n, int op) {
  std::vector<double> w(2 * n);
  for (int m = 0; m < n; ++m) {
    const long mp = signed_mode(m, n);
    if (op == OP_ROT) {  // half angle q/2 = 2 pi mp / (2n)
      double c, s;
      cos_sin(mp, 2L * n, &c, &s);
      w[2 * m] = s;
      w[2 * m + 1] = c;
    } else if (op == OP_WP) {
      // exp(i q) - 1 = -2 sin^2(q/2) + i 2 sin(q/2) cos(q/2): no cancellation at small q
      double ch, sh;
      cos_sin(mp, 2L * n, &ch, &sh);
      w[2 * m] = -2.0 * sh * sh;
      w[2 * m + 1] = 2.0 * sh * ch;
    } else if (op == OP_C) {  // sin q, exactly 0 at q = 0 and q = pi
      double c, s;
      cos_sin(mp, n, &c, &s);
      w[2 * m] = s;
      w[2 * m + 1] = 0.0;
    } else {  // MS
      w[2 * m] = 2.0 * M_PI * (double)mp / (double)n;
      w[2 * m + 1] = (n % 2 == 0 && 2 * m == n) ? 1.0 : 0.0;
    }
  }
  return w;
}

// ---------------------------------------------------------------------------
// plan
// ---------------------------------------------------------------------------
template <typename T>
struct Tables {
  cpx<T>* tw[3] = {nullptr, nullptr, nullptr};
  T* wave[3] = {nullptr, nullptr, nullptr};
};

struct fe_plan {
  fe_grid grid;
  fe_discretization disc;
  fe_scheme scheme;
  fe_plan_options opt;
  int device;
  hipStream_t stream;
  int op;
  bool displacement;  // WP/ROT: 3-component displacement form
  Dims d;
  int div_blocks;
  size_t partial_count;
  // workspace
  void* eps_ws = nullptr;
  void* R = nullptr;
  void* S = nullptr;
  double* partials = nullptr;
  double* partials2 = nullptr;
  double* red = nullptr;
  double* h_red = nullptr;  // pinned
  int* flag = nullptr;
  void* coef = nullptr;
  PhaseCoef<double>* coef64 = nullptr;
  Tables<float> t32;
  Tables<double> t64;
  size_t ws_bytes = 0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  hipEvent_t evc = nullptr;  // recorded after eta's copy to the host (the next passes run meanwhile)
  hipEvent_t tev[512] = {};  // pass timing pool (pairs)
  // mixed-precision refinement workspace (allocated on first use)
  void* dlt = nullptr;       // correction, 6 planes (plan precision)
  void* rfield = nullptr;    // strain residual of the anchor, 6 planes
  void* dsig_hi = nullptr;   // divergence of the anchor stress, 3 planes
  double* d64 = nullptr;     // float64 divergence / displacement, 3 planes
  cpx<double>* s64 = nullptr;  // float64 half spectra, 3 components
  void* dlt_alt = nullptr;     // second correction buffer (fused update + divergence)
  // six-component form, float64 work (allocated on first use): a strain, a
  // transform input/output and the half spectra (6 planes each); and for
  // float32 re-anchoring the anchor's divergence spectrum (6 half spectra of
  // the plan precision: conj(k).sigma at q and at its mirror)
  double* six64a = nullptr;
  double* six64b = nullptr;
  cpx<double>* six64s = nullptr;
  void* dbase6 = nullptr;
  // displacement form: second iterate and divergence buffers (allocated on first use)
  void* eps_alt = nullptr;
  void* R2 = nullptr;
  // conjugate gradients (allocated on first use): v, r, z, p, Q (3 planes
  // each), the sigma coefficient table and the device scalars
  void* cg = nullptr;
  void* coef_cg = nullptr;
  double* cgs = nullptr;
  // float32 conjugate gradients with float64 refinement: the displacement,
  // the residual and a conversion buffer (3 planes each), sigma table
  double* cg64 = nullptr;
  void* coef_cg64 = nullptr;
};

// Optional per-pass timing: HIP events recorded around each launch on the
// plan's stream; elapsed times are read back at synchronisation points.
struct PassTimer {
  fe_plan* p;
  bool on;
  int used = 0;
  static constexpr int kSlots = 256;
  int pass_of[kSlots];
  double sec[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int launches[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  PassTimer(fe_plan* plan, bool enabled) : p(plan), on(enabled) {}
  template <class F>
  void run(int pass, F&& f) {
    if (!on) {
      f();
      return;
    }
    if (used == kSlots) flush();
    (void)hipEventRecord(p->tev[2 * used], p->stream);
    f();
    (void)hipEventRecord(p->tev[2 * used + 1], p->stream);
    pass_of[used++] = pass;
  }
  void flush() {
    if (!on || used == 0) return;
    (void)hipEventSynchronize(p->tev[2 * used - 1]);
    for (int i = 0; i < used; ++i) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, p->tev[2 * i], p->tev[2 * i + 1]) == hipSuccess) sec[pass_of[i]] += ms * 1e-3;
      launches[pass_of[i]]++;
    }
    used = 0;
  }
};

static size_t elem_size(const fe_plan* p) { return p->opt.precision == FE_FP64 ? 8 : 4; }

extern "C" void fe_plan_options_default(fe_plan_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->struct_size = sizeof(fe_plan_options);
  o->precision = FE_FP32;
  o->max_iter = 1000;
  o->ref_rule = FE_REF_PAPER;
  o->ds_beta = 0.5;
  o->E0 = 0.0;
  o->nu0 = 0.25;
  o->check_every = 1;
  o->diverge_window = 50;
  o->timing = 0;
  o->refine = 1;
  o->hip_stream = nullptr;
  o->batch_launch = FE_BATCH_PER_PASS;
}

static hipError_t dmalloc(fe_plan* p, void** ptr, size_t bytes) {
  hipError_t e = hipMalloc(ptr, bytes);
  if (e == hipSuccess) p->ws_bytes += bytes;
  return e;
}

template <typename T>
static fe_status upload_tables(fe_plan* p, Tables<T>& t) {
  const int n[3] = {p->grid.nx, p->grid.ny, p->grid.nz};
  for (int a = 0; a < 3; ++a) {
    std::vector<double> tw = twiddles(n[a]);
    std::vector<double> wv = wave_table(n[a], p->op);
    std::vector<T> tw_t(tw.begin(), tw.end()), wv_t(wv.begin(), wv.end());
    HIP_TRY(dmalloc(p, (void**)&t.tw[a], tw_t.size() * sizeof(T)));
    HIP_TRY(dmalloc(p, (void**)&t.wave[a], wv_t.size() * sizeof(T)));
    HIP_TRY(hipMemcpy(t.tw[a], tw_t.data(), tw_t.size() * sizeof(T), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(t.wave[a], wv_t.data(), wv_t.size() * sizeof(T), hipMemcpyHostToDevice));
  }
  return FE_OK;
}

extern "C" fe_status fe_plan_create(fe_grid g, fe_discretization disc, fe_scheme scheme, const fe_plan_options* opt,
                                    fe_plan** out) {
  if (!out) return fail(FE_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  fe_plan_options o;
  fe_plan_options_default(&o);
  if (opt) {
    if (opt->struct_size != sizeof(fe_plan_options))
      return fail(FE_ERR_INVALID_ARG, "fe_plan_options.struct_size is %u, expected %zu", opt->struct_size,
                  sizeof(fe_plan_options));
    o = *opt;
  }
  if (disc < FE_GREEN_MS || disc > FE_GREEN_MS_SYMMETRIZED)
    return fail(FE_ERR_INVALID_ARG, "unknown discretization %d", (int)disc);
  if (scheme != FE_DIRECT && scheme != FE_ACCELERATED && scheme != FE_CONJUGATE_GRADIENT)
    return fail(FE_ERR_INVALID_ARG, "unknown scheme %d", (int)scheme);
  if (scheme == FE_CONJUGATE_GRADIENT && disc == FE_GREEN_MS_SYMMETRIZED)
    return fail(FE_ERR_UNSUPPORTED, "conjugate gradients need a projection operator (eq. (15)'s Nyquist rule is not)");
  if (o.precision != FE_FP32 && o.precision != FE_FP64)
    return fail(FE_ERR_INVALID_ARG, "unknown precision %d", (int)o.precision);
  if (o.max_iter < 0) return fail(FE_ERR_INVALID_ARG, "max_iter must be >= 0");
  if (o.check_every < 1) return fail(FE_ERR_INVALID_ARG, "check_every must be >= 1");
  if (o.diverge_window < 0) return fail(FE_ERR_INVALID_ARG, "diverge_window must be >= 0");
  if (o.ref_rule != FE_REF_PAPER && o.ref_rule != FE_REF_EXPLICIT)
    return fail(FE_ERR_INVALID_ARG, "unknown ref_rule %d", o.ref_rule);
  if (o.ref_rule == FE_REF_PAPER && scheme == FE_DIRECT && !(o.ds_beta > 0.0 && std::isfinite(o.ds_beta)))
    return fail(FE_ERR_INVALID_ARG, "ds_beta must be positive and finite");
  if (o.ref_rule == FE_REF_EXPLICIT &&
      !(std::isfinite(o.E0) && o.E0 > 0.0 && std::isfinite(o.nu0) && o.nu0 > -1.0 && o.nu0 < 0.5))
    return fail(FE_ERR_INVALID_ARG, "explicit reference needs E0 > 0 and -1 < nu0 < 0.5");
  const int n[3] = {g.nx, g.ny, g.nz};
  for (int a = 0; a < 3; ++a) {
    if (n[a] <= 0) return fail(FE_ERR_INVALID_ARG, "grid dimension %d is %d", a, n[a]);
    if (!(a == 2 ? supported_z_length(n[a]) : supported_length(n[a])))
      return fail(FE_ERR_UNSUPPORTED, "grid dimension %d = %d: need 2^a or 3*2^a in [4, 1024] (nz: or 1)", a, n[a]);
  }

  fe_plan* p = new fe_plan();
  p->grid = g;
  p->disc = disc;
  p->scheme = scheme;
  p->opt = o;
  p->stream = (hipStream_t)o.hip_stream;
  p->op = disc == FE_GREEN_MS    ? OP_MS
          : disc == FE_GREEN_WP  ? OP_WP
          : disc == FE_GREEN_ROT ? OP_ROT
          : disc == FE_GREEN_CENTERED ? OP_C
                                      : OP_MSS;
  p->displacement = p->op == OP_WP || p->op == OP_ROT;
  p->d = make_dims(g.nx, g.ny, g.nz);
  long long db = (p->d.N + kThreads - 1) / kThreads;
  p->div_blocks = (int)(db > kMaxReduceBlocks ? kMaxReduceBlocks : db);

  auto cleanup_fail = [&](fe_status s) {
    std::string keep = last_error_text();
    fe_plan_destroy(p);
    last_error_text() = keep;
    return s;
  };
  if (hipGetDevice(&p->device) != hipSuccess) return cleanup_fail(fail(FE_ERR_DEVICE, "no HIP device"));
  const size_t es = elem_size(p);
  const int ncomp = p->displacement ? 3 : 6;
  const long long N = p->d.N;
  const size_t spec = (size_t)spec_size(p->d);
  fe_status st;
  hipError_t e;
  if ((e = dmalloc(p, &p->R, (size_t)ncomp * N * es)) != hipSuccess)
    return cleanup_fail(fail(e == hipErrorOutOfMemory ? FE_ERR_OOM : FE_ERR_DEVICE, "workspace R: %s", hipGetErrorString(e)));
  if ((e = dmalloc(p, &p->S, (size_t)ncomp * spec * 2 * es)) != hipSuccess)
    return cleanup_fail(fail(e == hipErrorOutOfMemory ? FE_ERR_OOM : FE_ERR_DEVICE, "workspace S: %s", hipGetErrorString(e)));
  // partial sums: div/tau blocks x 7, and one per x-line block of the spectral eta
  const size_t lines = (size_t)p->d.Hp * g.ny;
  p->partial_count = (size_t)kMaxReduceBlocks * 7;
  if ((e = dmalloc(p, (void**)&p->partials, p->partial_count * sizeof(double))) != hipSuccess ||
      (e = dmalloc(p, (void**)&p->partials2, (lines + 1) * sizeof(double))) != hipSuccess ||
      (e = dmalloc(p, (void**)&p->red, 16 * sizeof(double))) != hipSuccess ||
      (e = dmalloc(p, (void**)&p->flag, sizeof(int))) != hipSuccess ||
      (e = dmalloc(p, &p->coef, 256 * sizeof(PhaseCoef<double>))) != hipSuccess ||
      (e = dmalloc(p, (void**)&p->coef64, 256 * sizeof(PhaseCoef<double>))) != hipSuccess)
    return cleanup_fail(fail(e == hipErrorOutOfMemory ? FE_ERR_OOM : FE_ERR_DEVICE, "workspace: %s", hipGetErrorString(e)));
  if (hipHostMalloc((void**)&p->h_red, 16 * sizeof(double), hipHostMallocDefault) != hipSuccess)
    return cleanup_fail(fail(FE_ERR_DEVICE, "pinned host buffer"));
  if ((st = upload_tables<float>(p, p->t32)) != FE_OK) return cleanup_fail(st);
  if ((st = upload_tables<double>(p, p->t64)) != FE_OK) return cleanup_fail(st);
  if (hipEventCreate(&p->ev0) != hipSuccess || hipEventCreate(&p->ev1) != hipSuccess ||
      hipEventCreateWithFlags(&p->evc, hipEventDisableTiming) != hipSuccess)
    return cleanup_fail(fail(FE_ERR_DEVICE, "event creation"));
  if (o.timing)
    for (int i = 0; i < 512; ++i)
      if (hipEventCreate(&p->tev[i]) != hipSuccess) return cleanup_fail(fail(FE_ERR_DEVICE, "event creation"));
  *out = p;
  return FE_OK;
}

template <typename T>
static void free_tables(Tables<T>& t) {
  for (int a = 0; a < 3; ++a) {
    if (t.tw[a]) (void)hipFree(t.tw[a]);
    if (t.wave[a]) (void)hipFree(t.wave[a]);
  }
}

extern "C" void fe_plan_destroy(fe_plan* p) {
  if (!p) return;
  (void)hipSetDevice(p->device);
  void* bufs[] = {p->eps_ws, p->R,      p->S,       p->partials, p->partials2, p->red,     p->flag,   p->coef,
                  p->coef64, p->dlt,    p->rfield,  p->dsig_hi,  p->d64,       p->s64,     p->dlt_alt, p->eps_alt,
                  p->R2,     p->cg,     p->coef_cg, p->cgs,      p->cg64,      p->coef_cg64, p->six64a,  p->six64b,
                  p->six64s, p->dbase6};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  free_tables(p->t32);
  free_tables(p->t64);
  if (p->h_red) (void)hipHostFree(p->h_red);
  if (p->ev0) (void)hipEventDestroy(p->ev0);
  if (p->ev1) (void)hipEventDestroy(p->ev1);
  if (p->evc) (void)hipEventDestroy(p->evc);
  for (hipEvent_t e : p->tev)
    if (e) (void)hipEventDestroy(e);
  delete p;
}

extern "C" size_t fe_plan_workspace_bytes(const fe_plan* p) { return p ? p->ws_bytes : 0; }

// ---------------------------------------------------------------------------
// solve
// ---------------------------------------------------------------------------
struct RefMedium {
  double lam0, mu0, kap0;
};

static RefMedium reference_medium(const fe_plan_options& o, fe_scheme scheme, const fe_materials& m) {
  RefMedium r;
  if (o.ref_rule == FE_REF_EXPLICIT) {
    const double E = o.E0, nu = o.nu0;
    r.lam0 = E * nu / ((1 + nu) * (1 - 2 * nu));
    r.mu0 = E / (2 * (1 + nu));
  } else {
    double kmin = INFINITY, kmax = -INFINITY, mmin = INFINITY, mmax = -INFINITY;
    for (int i = 0; i < m.n_phases; ++i) {
      const double E = m.E[i], nu = m.nu[i];
      const double lam = E * nu / ((1 + nu) * (1 - 2 * nu)), mu = E / (2 * (1 + nu));
      const double kap = lam + 2.0 * mu / 3.0;
      kmin = std::fmin(kmin, kap);
      kmax = std::fmax(kmax, kap);
      mmin = std::fmin(mmin, mu);
      mmax = std::fmax(mmax, mu);
    }
    double k0, m0;
    if (scheme != FE_DIRECT) {  // eq. (17); conjugate gradients take the same medium
      k0 = std::sqrt(kmin * kmax);
      m0 = std::sqrt(mmin * mmax);
    } else {  // eq. (18)
      k0 = o.ds_beta * (kmin + kmax);
      m0 = o.ds_beta * (mmin + mmax);
    }
    r.mu0 = m0;
    r.lam0 = k0 - 2.0 * m0 / 3.0;
  }
  r.kap0 = r.lam0 + 2.0 * r.mu0 / 3.0;
  return r;
}

static std::vector<PhaseCoef<double>> phase_coefs(const fe_materials& m, const RefMedium& r) {
  std::vector<PhaseCoef<double>> c(m.n_phases);
  for (int i = 0; i < m.n_phases; ++i) {
    const double E = m.E[i], nu = m.nu[i];
    const double lam = E * nu / ((1 + nu) * (1 - 2 * nu)), mu = E / (2 * (1 + nu));
    const double kap = lam + 2.0 * mu / 3.0;
    c[i].lam = lam;
    c[i].mu = mu;
    c[i].dlam = lam - r.lam0;
    c[i].dmu = mu - r.mu0;
    c[i].ak = 2.0 * r.kap0 / (kap + r.kap0);
    c[i].am = 2.0 * r.mu0 / (mu + r.mu0);
    c[i].pad0 = c[i].pad1 = 0.0;
  }
  return c;
}

static fe_status validate_materials(const fe_materials& m) {
  if (m.n_phases < 1 || m.n_phases > 256) return fail(FE_ERR_INVALID_ARG, "n_phases must be in [1, 256]");
  if (!m.E || !m.nu) return fail(FE_ERR_INVALID_ARG, "materials arrays are NULL");
  for (int i = 0; i < m.n_phases; ++i) {
    if (!(std::isfinite(m.E[i]) && m.E[i] > 0.0))
      return fail(FE_ERR_INVALID_ARG, "phase %d: Young's modulus must be finite and > 0", i);
    if (!(std::isfinite(m.nu[i]) && m.nu[i] > -1.0 && m.nu[i] < 0.5))
      return fail(FE_ERR_INVALID_ARG, "phase %d: Poisson ratio must be in (-1, 0.5)", i);
  }
  return FE_OK;
}

// Frobenius norm of a symmetric tensor given in Voigt order (off-diagonals twice).
static double frob(const double* s) {
#pragma clang fp contract(off)  // the roundings of the device's eta in batched solves
  return std::sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2] + 2.0 * (s[3] * s[3] + s[4] * s[4] + s[5] * s[5]));
}

template <typename T>
static const Tables<T>& tables(const fe_plan* p);
template <>
const Tables<float>& tables<float>(const fe_plan* p) { return p->t32; }
template <>
const Tables<double>& tables<double>(const fe_plan* p) { return p->t64; }

template <typename T>
static Tables<T>& tables_mut(fe_plan* p);
template <>
Tables<float>& tables_mut<float>(fe_plan* p) { return p->t32; }
template <>
Tables<double>& tables_mut<double>(fe_plan* p) { return p->t64; }

template <typename T>
static WaveTables<T> wave_tables(const fe_plan* p) {
  const Tables<T>& t = tables<T>(p);
  return WaveTables<T>{t.wave[0], t.wave[1], t.wave[2]};
}

// float64 work buffers of the six-component form (verification, re-anchoring)
static fe_status six64_workspace(fe_plan* p) {
  const size_t N = (size_t)p->d.N, spec = (size_t)spec_size(p->d);
  if (!p->six64a) HIP_TRY(dmalloc(p, (void**)&p->six64a, 6 * N * sizeof(double)));
  if (!p->six64b) HIP_TRY(dmalloc(p, (void**)&p->six64b, 6 * N * sizeof(double)));
  if (!p->six64s) HIP_TRY(dmalloc(p, (void**)&p->six64s, 6 * spec * sizeof(cpx<double>)));
  return FE_OK;
}

// eta and <sigma> of the current strain (float64 arithmetic from a strain of
// storage type TS), via the spectral 6-component path for MS or the
// corner/backward stencil otherwise.  Requires a float64 workspace for MS when
// TS is float (allocated and released here).
template <typename TS>
static fe_status verify_fp64(fe_plan* p, const TS* eps, const uint8_t* phase, double* eta_out) {
  hipStream_t s = p->stream;
  const Dims d = p->d;
  if (p->displacement) {
    const int nb = launch_verify_div<TS>(eps, phase, p->coef64, p->partials, d, p->op, s);
    launch_reduce(p->partials, nb, 7, p->red, s);
    HIP_TRY(hipMemcpyAsync(p->h_red, p->red, 7 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    double ms[6];
    for (int i = 0; i < 6; ++i) ms[i] = p->h_red[1 + i] / (double)d.N;
    *eta_out = std::sqrt(p->h_red[0] / (double)d.N) / frob(ms);
    return FE_OK;
  }
  if (six64_workspace(p) != FE_OK) {  // no room for the float64 work: no verification
    (void)hipGetLastError();
    *eta_out = NAN;
    return FE_OK;
  }
  double* e64 = p->six64a;
  double* r64 = p->six64b;
  cpx<double>* s64 = p->six64s;
  Launch<double>::convert_to(e64, eps, sizeof(TS) == 8, 6 * d.N, s);
  Launch<double>::tau6(e64, phase, p->coef64, r64, 1, p->partials, p->div_blocks, d, s);
  launch_reduce(p->partials, p->div_blocks, 7, p->red, s);
  const Tables<double>& t = p->t64;
  Launch<double>::zr2c(r64, s64, 6, d, t.tw[2], s);
  Launch<double>::yfft(s64, 6, d, t.tw[1], 0, s);
  const int nblk = Launch<double>::xeta6(s64, d, t.tw[0], wave_tables<double>(p), p->partials2, p->op, s);
  launch_reduce(p->partials2, nblk, 1, p->red + 8, s);
  HIP_TRY(hipMemcpyAsync(p->h_red, p->red, 9 * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  double ms[6];
  for (int i = 0; i < 6; ++i) ms[i] = p->h_red[1 + i] / (double)d.N;
  *eta_out = std::sqrt(p->h_red[8]) / ((double)d.N * frob(ms));
  return FE_OK;
}

// Conjugate gradients (displacement form, WP and ROT).  The iterate is the
// strain eps_bar + grad v of a corner displacement v; the residual r is the
// corner divergence of sigma of that strain (the quantity eta measures); the
// preconditioner is the reference medium's operator, inverted by the same
// transform passes as the fixed-point schemes (z, y, x with the Green step, y,
// z).  These are the iterates of conjugate gradients on the strain in the
// C0-weighted inner product.  The sign of the divergence stencil cancels in
// alpha and beta.  Every scalar stays on the device; the host reads |r|^2 and
// the mean stress once per iteration while the next preconditioner step runs.
// A float32 residual drifts from the true one: when the recurrence says
// eta <= tol the true residual is recomputed, and the iteration restarts from
// it if it is not there (stopping when a restart gains less than 2x).
template <typename T>
static fe_status solve_cg(fe_plan* p, const uint8_t* phase, const std::vector<PhaseCoef<T>>& cT,
                          const std::vector<PhaseCoef<double>>& c64, const PhaseCoef<T>* coef, const GreenConst<T>& g,
                          const double* macro, T* eps, double tol, fe_result* out) {
  hipStream_t s = p->stream;
  const Dims d = p->d;
  const long long N = d.N, n3 = 3 * N;
  const Tables<T>& tb = tables<T>(p);
  const WaveTables<T> wt = wave_tables<T>(p);
  std::vector<PhaseCoef<T>> cs(cT);  // "tau" of this table is sigma: the fused launch writes div sigma
  for (auto& c : cs) {
    c.dlam = c.lam;
    c.dmu = c.mu;
  }
  if (!p->coef_cg) HIP_TRY(dmalloc(p, &p->coef_cg, 256 * sizeof(PhaseCoef<double>)));
  if (!p->cgs) HIP_TRY(dmalloc(p, (void**)&p->cgs, 32 * sizeof(double)));
  if (!p->cg) HIP_TRY(dmalloc(p, &p->cg, 5 * (size_t)n3 * sizeof(T)));
  HIP_TRY(hipMemcpyAsync(p->coef_cg, cs.data(), cs.size() * sizeof(PhaseCoef<T>), hipMemcpyHostToDevice, s));
  const PhaseCoef<T>* csig = static_cast<const PhaseCoef<T>*>(p->coef_cg);
  T* v = static_cast<T*>(p->cg);
  T* r = v + n3;
  T* z = r + n3;
  T* pd = z + n3;
  T* Q = pd + n3;
  cpx<T>* S = static_cast<cpx<T>*>(p->S);
  double* cgs = p->cgs;
  GreenConst<T> g0 = g;  // grad p alone: no applied strain
  for (int i = 0; i < 6; ++i) g0.macro[i] = T(0);
  HIP_TRY(hipMemsetAsync(v, 0, (size_t)n3 * sizeof(T), s));
  HIP_TRY(hipMemsetAsync(cgs, 0, 32 * sizeof(double), s));
  // float32 with refinement: the displacement is v64 + v, v64 in float64;
  // every true residual folds v into v64 and is formed in float64
  const bool refine64 = sizeof(T) == 4 && p->opt.refine;
  double *v64 = nullptr, *R64 = nullptr, *t64 = nullptr;
  const PhaseCoef<double>* csig64 = nullptr;
  GreenConst<double> g64;
  std::memset(&g64, 0, sizeof g64);
  if (refine64) {
    if (!p->cg64) HIP_TRY(dmalloc(p, (void**)&p->cg64, 9 * (size_t)N * sizeof(double)));
    if (!p->coef_cg64) HIP_TRY(dmalloc(p, &p->coef_cg64, 256 * sizeof(PhaseCoef<double>)));
    std::vector<PhaseCoef<double>> cs64(c64);
    for (auto& c : cs64) {
      c.dlam = c.lam;
      c.dmu = c.mu;
    }
    HIP_TRY(hipMemcpyAsync(p->coef_cg64, cs64.data(), cs64.size() * sizeof(PhaseCoef<double>),
                           hipMemcpyHostToDevice, s));
    csig64 = static_cast<const PhaseCoef<double>*>(p->coef_cg64);
    v64 = p->cg64;
    R64 = v64 + n3;
    t64 = R64 + n3;
    HIP_TRY(hipMemsetAsync(v64, 0, (size_t)n3 * sizeof(double), s));
    for (int i = 0; i < 6; ++i) g64.macro[i] = macro[i];  // the strain update in float64 uses eps_bar only
  }

  // D = div sigma(eps_bar + grad v) with |D|^2 and the sums of sigma into
  // cgs[3], cgs[10..15]; the strain goes to eps (free until the end).  With
  // refinement: v is folded into v64 (v = 0 after) and D = float(R64).
  auto true_residual = [&](T* D) {
    if (refine64) {
      Launch<double>::convert_to(t64, v, 0, n3, s);
      Launch<double>::axpy(v64, t64, n3, s);
      (void)hipMemsetAsync(v, 0, (size_t)n3 * sizeof(T), s);
      int nb = Launch<double>::update_div(v64, v64, nullptr, phase, csig64, g64, nullptr, R64, nullptr, p->partials,
                                          d, p->op, 0, s);
      launch_reduce(p->partials, nb, 7, cgs + 16, s);
      nb = Launch<double>::dot(R64, R64, n3, p->partials, s);
      launch_reduce(p->partials, nb, 1, cgs + 16, s);
      launch_cg_restart(cgs, s);
      Launch<T>::convert_to(D, R64, 1, n3, s);
      return;
    }
    const int nb = Launch<T>::update_div(v, v, eps, phase, csig, g, nullptr, D, nullptr, p->partials, d, p->op, 0, s);
    launch_reduce(p->partials, nb, 7, cgs + 16, s);
    launch_cg_restart(cgs, s);
  };
  auto precond = [&]() {  // z = K0^-1 r (up to sign) and rho = r.z
    Launch<T>::zr2c(r, S, 3, d, tb.tw[2], s);
    Launch<T>::yfft(S, 3, d, tb.tw[1], 0, s);
    Launch<T>::xgreen3(S, d, tb.tw[0], wt, g, p->op, s);
    Launch<T>::yfft(S, 3, d, tb.tw[1], 1, s);
    Launch<T>::zc2r(S, z, 3, d, tb.tw[2], s);
    const int nb = Launch<T>::dot(r, z, n3, p->partials, s);
    launch_reduce(p->partials, nb, 1, cgs + 0, s);
  };
  // eta from |r|^2 and the voxel sums of sigma (host copy of cgs[3], cgs[10..15])
  double mean[6] = {0, 0, 0, 0, 0, 0};
  auto eta_of = [&]() {
    for (int i = 0; i < 6; ++i) mean[i] = p->h_red[1 + i] / (double)N;
    return std::sqrt(p->h_red[0] / (double)N) / frob(mean);
  };
  auto record = [&](int kk, double e) {
    if (kk >= out->history_capacity) return;
    if (out->eta_history) out->eta_history[kk] = e;
    if (out->mean_stress_history)
      for (int i = 0; i < 6; ++i) out->mean_stress_history[6 * kk + i] = mean[i];
  };
  auto fetch = [&]() -> fe_status {
    HIP_TRY(hipMemcpyAsync(p->h_red, cgs + 3, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(p->h_red + 1, cgs + 10, 6 * sizeof(double), hipMemcpyDeviceToHost, s));
    return FE_OK;
  };

  // r = D(v), z = K0^-1 r, p = z: the start, and every restart of the
  // refined iteration below
  auto start = [&]() -> fe_status {
    true_residual(r);
    fe_status fs = fetch();
    if (fs != FE_OK) return fs;
    HIP_TRY(hipEventRecord(p->evc, s));
    precond();
    Launch<T>::cg_dir(pd, z, n3, cgs, 1, s);
    HIP_TRY(hipEventSynchronize(p->evc));
    return FE_OK;
  };
  HIP_TRY(hipEventRecord(p->ev0, s));
  {
    fe_status fs = start();
    if (fs != FE_OK) return fs;
  }
  const int max_iter = p->opt.max_iter;
  fe_status status = FE_NOT_CONVERGED;
  double eta = eta_of(), restart_eta = INFINITY, best = INFINITY;
  int k = 0, best_k = 0;
  // With refinement the float64 residual of v64 + v reaching target is not
  // the end: the float32 strain returned carries its own rounding, which
  // adds to that residual.  If the strain does not verify to tol, the
  // iteration goes on towards half the target (at most four times, and only
  // while the verified eta still falls by 10%).
  double target = tol, ev = INFINITY, ev_last = INFINITY, eta_end = INFINITY;
  float ms_elapsed = 0.f;
  for (int lowered = 0;; ++lowered) {
  for (;; ++k) {
    record(k, eta);
    if (!std::isfinite(eta)) {
      status = FE_DIVERGED;
      break;
    }
    // The recursive residual says converged, or has not gained 5% in 20
    // iterations: compare with the true residual.  A gap of more than 10%
    // is rounding drift (float32 storage): restart from the true residual,
    // unless the last restart gained less than a factor 2 (storage floor).
    bool stalled = false;
    if (eta < 0.95 * best) {
      best = eta;
      best_k = k;
    } else if (k - best_k >= 20) {
      stalled = true;
    }
    if (eta <= target || stalled) {
      const double eta_rec = eta;
      true_residual(Q);  // Q is free until the next step
      fe_status fs = fetch();
      if (fs != FE_OK) return fs;
      HIP_TRY(hipStreamSynchronize(s));
      eta = eta_of();
      record(k, eta);
      if (eta <= target) {
        status = FE_OK;
        break;
      }
      best = std::fmin(best, eta);
      best_k = k;
      if (std::fabs(eta - eta_rec) > 0.1 * eta_rec) {
        if (!(eta < 0.5 * restart_eta)) break;  // storage floor: a restart no longer gains
        restart_eta = eta;
        best = eta;
        true_residual(r);
        precond();
        Launch<T>::cg_dir(pd, z, n3, cgs, 1, s);
      }
    }
    if (k >= max_iter) break;
    // Q = div sigma(grad p) = -K p (up to the stencil's sign) with p.Q and the sums of sigma
    int nb = Launch<T>::update_div(pd, pd, nullptr, phase, csig, g0, nullptr, Q, nullptr, p->partials, d, p->op, 0, s);
    launch_reduce(p->partials, nb, 7, cgs + 16, s);
    nb = Launch<T>::cg_step(v, pd, r, Q, n3, cgs, p->partials, s);
    launch_reduce(p->partials, nb, 1, cgs + 3, s);
    fe_status fs = fetch();
    if (fs != FE_OK) return fs;
    HIP_TRY(hipEventRecord(p->evc, s));
    precond();  // queued while the host reads eta^(k+1)
    Launch<T>::cg_dir(pd, z, n3, cgs, 0, s);
    HIP_TRY(hipEventSynchronize(p->evc));
    eta = eta_of();
    HIP_TRY(hipGetLastError());
  }
  // the strain eps_bar + grad v, its residual and mean stress
  true_residual(r);
  {
    fe_status fs = fetch();
    if (fs != FE_OK) return fs;
  }
  if (refine64) {
    // eps: the strain formed in float64 and rounded once (a float copy of the
    // displacement would put its rounding, |v| times 6e-8, into the gradient).
    // R64 and t64 (6 contiguous float64 planes) take the strain, r and z (3
    // float64 planes' worth) the divergence that the launch also writes.
    double* e64 = R64;
    Launch<double>::update_div(v64, v64, e64, phase, csig64, g64, nullptr, reinterpret_cast<double*>(r), nullptr,
                               p->partials, d, p->op, 0, s);
    Launch<T>::convert_to(eps, e64, 1, 6 * N, s);
  }
  HIP_TRY(hipEventRecord(p->ev1, s));
  HIP_TRY(hipEventSynchronize(p->ev1));
  eta_end = eta_of();
  HIP_TRY(hipEventElapsedTime(&ms_elapsed, p->ev0, p->ev1));
  ev = eta_end;
  if (sizeof(T) == 4) {
    fe_status vs = verify_fp64<T>(p, eps, phase, &ev);
    if (vs != FE_OK) return vs;
  }
  if (!(refine64 && status == FE_OK && !(ev <= tol))) break;
  // the float32 strain returned must itself meet tol (its storage floor)
  status = FE_NOT_CONVERGED;
  if (lowered >= 4 || k >= max_iter || !(ev < 0.9 * ev_last)) break;
  ev_last = ev;
  target *= 0.5;
  {
    fe_status fs = start();  // r and z were overwritten by the strain above
    if (fs != FE_OK) return fs;
  }
  eta = eta_of();
  best = eta;
  best_k = k;
  restart_eta = INFINITY;
  }
  for (int i = 0; i < 8; ++i) {
    out->pass_seconds[i] = 0.0;
    out->pass_launches[i] = 0;
  }
  out->refinements = 0;
  if (out->stress) Launch<T>::stress(eps, phase, coef, static_cast<T*>(out->stress), N, s);
  HIP_TRY(hipStreamSynchronize(s));
  out->iterations = k;
  out->eta = status == FE_OK ? eta : eta_end;
  out->eta_verify_fp64 = ev;
  out->seconds = ms_elapsed * 1e-3;
  for (int i = 0; i < 6; ++i) out->mean_stress[i] = mean[i];
  if (status == FE_NOT_CONVERGED)
    fail(status, "not converged after %d iterations (eta = %.3e, tol = %.3e)", k, eta_end, tol);
  else if (status == FE_DIVERGED)
    fail(status, "diverged at iteration %d (eta = %.3e)", k, eta);
  return status;
}

// Conjugate gradients in the six-component form (MS, C): the iterate is the
// strain eps = eps_bar + e with e compatible and of zero mean; with
// B(x) = G' * (C : x) (a C0-orthogonal projection after C, self-adjoint and
// positive in <a, b> = sum_x a : C0 : b on compatible fields) the fluctuation
// solves B(e) = -B(eps_bar).  Per iteration: B(p) by the transform passes
// with no applied strain, <p, B(p)>, the step, the direction, and eta^k of
// eps (eq. (43), spectral).  The scalars stay on the device; the host reads
// eta.  Float32 plans run in float32 (no refinement): no 5% gain in eta over
// 100 iterations ends the run at the float32 floor (FE_NOT_CONVERGED).
template <typename T>
static fe_status solve_cg6(fe_plan* p, const uint8_t* phase, const PhaseCoef<T>* coef, const GreenConst<T>& g,
                           const RefMedium& ref, const double* macro, T* eps, double tol, fe_result* out) {
  hipStream_t s = p->stream;
  const Dims d = p->d;
  const long long N = d.N, n6 = 6 * N;
  const Tables<T>& tb = tables<T>(p);
  const WaveTables<T> wt = wave_tables<T>(p);
  if (!p->cgs) HIP_TRY(dmalloc(p, (void**)&p->cgs, 32 * sizeof(double)));
  if (!p->cg) HIP_TRY(dmalloc(p, &p->cg, 3 * (size_t)n6 * sizeof(T)));
  T* r = static_cast<T*>(p->cg);
  T* pd = r + n6;
  T* Q = pd + n6;
  T* R = static_cast<T*>(p->R);
  cpx<T>* S = static_cast<cpx<T>*>(p->S);
  double* cgs = p->cgs;
  GreenConst<T> gz = g;  // B(x): no applied strain
  for (int i = 0; i < 6; ++i) gz.macro[i] = T(0);
  // Qout = (negate ? B(x) : -B(x)), dst = <dotx, Qout> (dotx NULL: <Qout, Qout>)
  auto apply_b = [&](const T* x, T* Qout, const T* dotx, int negate, double* dst) {
    Launch<T>::tau6(x, phase, coef, R, 1, nullptr, p->div_blocks, d, s);
    Launch<T>::zr2c(R, S, 6, d, tb.tw[2], s);
    Launch<T>::yfft(S, 6, d, tb.tw[1], 0, s);
    Launch<T>::xgreen6(S, d, tb.tw[0], wt, gz, p->op, s);
    Launch<T>::yfft(S, 6, d, tb.tw[1], 1, s);
    Launch<T>::zc2r(S, R, 6, d, tb.tw[2], s);
    const int nb = Launch<T>::cg6_take(R, Qout, dotx, negate, d, ref.lam0, ref.mu0, p->partials, s);
    launch_reduce(p->partials, nb, 1, dst, s);
  };
  double mean[6] = {0, 0, 0, 0, 0, 0};
  auto eta_now = [&](double* e) -> fe_status {
    Launch<T>::tau6(eps, phase, coef, R, 1, p->partials, p->div_blocks, d, s);
    launch_reduce(p->partials, p->div_blocks, 7, p->red, s);
    Launch<T>::zr2c(R, S, 6, d, tb.tw[2], s);
    Launch<T>::yfft(S, 6, d, tb.tw[1], 0, s);
    const int xblk = Launch<T>::xeta6(S, d, tb.tw[0], wt, p->partials2, p->op, s);
    launch_reduce(p->partials2, xblk, 1, p->red + 8, s);
    HIP_TRY(hipMemcpyAsync(p->h_red, p->red, 9 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int i = 0; i < 6; ++i) mean[i] = p->h_red[1 + i] / (double)N;
    *e = std::sqrt(p->h_red[8]) / ((double)N * frob(mean));
    return FE_OK;
  };
  auto record = [&](int kk, double e) {
    if (kk >= out->history_capacity) return;
    if (out->eta_history) out->eta_history[kk] = e;
    if (out->mean_stress_history)
      for (int i = 0; i < 6; ++i) out->mean_stress_history[6 * kk + i] = mean[i];
  };
  const auto host_t0 = std::chrono::steady_clock::now();
  HIP_TRY(hipMemsetAsync(cgs, 0, 32 * sizeof(double), s));
  Launch<T>::fill_macro(eps, N, macro, s);
  apply_b(eps, r, nullptr, 0, cgs + 0);  // r = -B(eps_bar), <r, r>
  Launch<T>::cg_dir(pd, r, n6, cgs, 1, s);
  fe_status status = FE_NOT_CONVERGED;
  double eta = NAN, best = INFINITY;
  int k = 0, best_k = 0;
  for (;; ++k) {
    fe_status es = eta_now(&eta);
    if (es != FE_OK) return es;
    record(k, eta);
    if (!std::isfinite(eta)) {
      status = FE_DIVERGED;
      break;
    }
    if (eta <= tol) {
      status = FE_OK;
      break;
    }
    if (k >= p->opt.max_iter) break;
    if (eta < 0.95 * best) {
      best = eta;
      best_k = k;
    } else if (sizeof(T) == 4 && k - best_k >= 100) {
      break;  // float32 floor
    }
    apply_b(pd, Q, pd, 1, cgs + 16);  // Q = B(p), <p, Q>
    const int nb = Launch<T>::cg6_step(eps, pd, r, Q, N, ref.lam0, ref.mu0, cgs, p->partials, s);
    launch_reduce(p->partials, nb, 1, cgs + 0, s);
    Launch<T>::cg_dir(pd, r, n6, cgs, 0, s);
    HIP_TRY(hipGetLastError());
  }
  HIP_TRY(hipStreamSynchronize(s));
  const double seconds =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - host_t0).count();
  for (int i = 0; i < 8; ++i) {
    out->pass_seconds[i] = 0.0;
    out->pass_launches[i] = 0;
  }
  out->refinements = 0;
  if (out->stress) Launch<T>::stress(eps, phase, coef, static_cast<T*>(out->stress), N, s);
  double ev = eta;
  if (sizeof(T) == 4) {
    fe_status vs = verify_fp64<T>(p, eps, phase, &ev);
    if (vs != FE_OK) return vs;
  }
  HIP_TRY(hipStreamSynchronize(s));
  out->iterations = k;
  out->eta = eta;
  out->eta_verify_fp64 = ev;
  out->seconds = seconds;
  for (int i = 0; i < 6; ++i) out->mean_stress[i] = mean[i];
  if (status == FE_NOT_CONVERGED)
    fail(status, "not converged after %d iterations (eta = %.3e, tol = %.3e)", k, eta, tol);
  else if (status == FE_DIVERGED)
    fail(status, "diverged at iteration %d (eta = %.3e)", k, eta);
  return status;
}

template <typename T>
static fe_status solve_impl(fe_plan* p, const uint8_t* phase, const fe_materials& mat, const double* macro, double tol,
                            const void* strain_init, fe_result* out) {
  hipStream_t s = p->stream;
  const Dims d = p->d;
  const long long N = d.N;
  const Tables<T>& tb = tables<T>(p);
  const WaveTables<T> wt = wave_tables<T>(p);

  // per-phase constants (float64 on the host, rounded to T for the kernels)
  const RefMedium ref = reference_medium(p->opt, p->scheme, mat);
  std::vector<PhaseCoef<double>> c64 = phase_coefs(mat, ref);
  std::vector<PhaseCoef<T>> cT(c64.size());
  for (size_t i = 0; i < c64.size(); ++i) {
    cT[i].lam = T(c64[i].lam);
    cT[i].mu = T(c64[i].mu);
    cT[i].dlam = T(c64[i].dlam);
    cT[i].dmu = T(c64[i].dmu);
    cT[i].ak = T(c64[i].ak);
    cT[i].am = T(c64[i].am);
    cT[i].pad0 = cT[i].pad1 = T(0);
  }
  HIP_TRY(hipMemcpyAsync(p->coef, cT.data(), cT.size() * sizeof(PhaseCoef<T>), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(p->coef64, c64.data(), c64.size() * sizeof(PhaseCoef<double>), hipMemcpyHostToDevice, s));
  const PhaseCoef<T>* coef = static_cast<const PhaseCoef<T>*>(p->coef);

  GreenConst<T> g;
  g.lam0 = T(ref.lam0);
  g.mu0 = T(ref.mu0);
  g.cr = T((ref.lam0 + ref.mu0) / (ref.lam0 + 2.0 * ref.mu0));
  g.s1 = T(1.0 / (2.0 * ref.mu0));
  g.s2 = T(ref.lam0 / (2.0 * ref.mu0 * (3.0 * ref.lam0 + 2.0 * ref.mu0)));
  g.inv_n = T(1.0 / (double)N);
  for (int i = 0; i < 6; ++i) g.macro[i] = T(macro[i]);

  // phase labels must index the table
  HIP_TRY(hipMemsetAsync(p->flag, 0, sizeof(int), s));
  Launch<T>::check_phase(phase, N, mat.n_phases, p->flag, s);
  int hflag = 0;
  HIP_TRY(hipMemcpyAsync(&hflag, p->flag, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (hflag) return fail(FE_ERR_INVALID_ARG, "phase map holds a label >= n_phases (%d)", mat.n_phases);

  T* eps = static_cast<T*>(out->strain);
  if (!eps) {
    if (!p->eps_ws) HIP_TRY(dmalloc(p, &p->eps_ws, 6 * (size_t)N * sizeof(T)));
    eps = static_cast<T*>(p->eps_ws);
  }
  if (p->scheme == FE_CONJUGATE_GRADIENT)
    return p->displacement ? solve_cg<T>(p, phase, cT, c64, coef, g, macro, eps, tol, out)
                           : solve_cg6<T>(p, phase, coef, g, ref, macro, eps, tol, out);
  if (strain_init) {
    if (strain_init != eps)
      HIP_TRY(hipMemcpyAsync(eps, strain_init, 6 * (size_t)N * sizeof(T), hipMemcpyDeviceToDevice, s));
  } else {
    Launch<T>::fill_macro(eps, N, macro, s);
  }

  T* R = static_cast<T*>(p->R);
  cpx<T>* S = static_cast<cpx<T>*>(p->S);
  T* R2 = nullptr;  // displacement form: the fused update writes the next divergence here
  if (p->displacement) {
    if (!p->R2) HIP_TRY(dmalloc(p, &p->R2, 3 * (size_t)N * sizeof(T)));
    if (!p->eps_alt) HIP_TRY(dmalloc(p, &p->eps_alt, 6 * (size_t)N * sizeof(T)));
    R2 = static_cast<T*>(p->R2);
  }
  const int ncomp = p->displacement ? 3 : 6;
  const int accel = p->scheme == FE_ACCELERATED;
  const int max_iter = p->opt.max_iter;
  const int every = p->opt.check_every;

  const bool can_refine = p->opt.refine && sizeof(T) == 4;
  GreenConst<T> gz = g;  // the correction of an anchored iteration: no applied strain (the residual field replaces it)
  for (int i = 0; i < 6; ++i) gz.macro[i] = T(0);
  GreenConst<double> g64;
  g64.lam0 = ref.lam0;
  g64.mu0 = ref.mu0;
  g64.cr = (ref.lam0 + ref.mu0) / (ref.lam0 + 2.0 * ref.mu0);
  g64.s1 = 1.0 / (2.0 * ref.mu0);
  g64.s2 = ref.lam0 / (2.0 * ref.mu0 * (3.0 * ref.lam0 + 2.0 * ref.mu0));
  g64.inv_n = 1.0 / (double)N;
  for (int i = 0; i < 6; ++i) g64.macro[i] = macro[i];

  // State: without an anchor the iterate is eps itself; with an anchor the
  // strain is eps + it, where it = correction (it starts at 0 at each re-anchor)
  // and the anchor's strain residual rf and stress divergence dbase come from
  // float64 arithmetic.
  T* it = eps;
  T* nxt = static_cast<T*>(p->eps_alt);  // the fused update writes the next iterate here, then they swap
  const T* rf = nullptr;
  const T* dbase = nullptr;
  double mean_hi[6] = {0, 0, 0, 0, 0, 0};
  bool anchored = false;
  int refinements = 0;
  bool have_D = false;  // R holds the divergence of the current iterate and partials its sums
  int nb_D = 0;
  // without an anchor the strain must sit in eps before float64 work reads it
  auto sync_iterate = [&]() -> fe_status {
    if (!anchored && it != eps) {
      HIP_TRY(hipMemcpyAsync(eps, it, 6 * (size_t)N * sizeof(T), hipMemcpyDeviceToDevice, s));
      nxt = it;
      it = eps;
    }
    return FE_OK;
  };

  // six-component form: the anchor's iterate e_hi = eps_bar - G' tau(eps)
  // and its residual r = e_hi - eps, the mean and the divergence spectrum of
  // sigma(eps), all from float64 arithmetic; the float32 iterations then
  // solve for the correction delta with r in place of the applied strain
  // (eqs. (9), (16) are affine in the iterate) and eta adds the anchor's
  // divergence spectrum before the square.
  auto reanchor6 = [&]() -> fe_status {
    const size_t spec = (size_t)spec_size(d);
    fe_status ss = six64_workspace(p);
    if (ss != FE_OK) return ss;
    if (!p->dlt) {
      HIP_TRY(dmalloc(p, &p->dlt, 6 * (size_t)N * sizeof(T)));
      HIP_TRY(dmalloc(p, &p->rfield, 6 * (size_t)N * sizeof(T)));
      HIP_TRY(dmalloc(p, &p->dbase6, 6 * spec * sizeof(cpx<T>)));
    }
    if (anchored) Launch<T>::axpy(eps, it, 6 * N, s);
    double* e64 = p->six64a;
    double* w64 = p->six64b;
    cpx<double>* S64 = p->six64s;
    const Tables<double>& t = p->t64;
    const WaveTables<double> wt64 = wave_tables<double>(p);
    Launch<double>::convert_to(e64, eps, sizeof(T) == 8, 6 * N, s);
    Launch<double>::tau6(e64, phase, p->coef64, w64, 0, nullptr, p->div_blocks, d, s);
    Launch<double>::zr2c(w64, S64, 6, d, t.tw[2], s);
    Launch<double>::yfft(S64, 6, d, t.tw[1], 0, s);
    Launch<double>::xgreen6(S64, d, t.tw[0], wt64, g64, p->op, s);
    Launch<double>::yfft(S64, 6, d, t.tw[1], 1, s);
    Launch<double>::zc2r(S64, w64, 6, d, t.tw[2], s);
    launch_residual6<T>(w64, eps, static_cast<T*>(p->rfield), d, s);
    Launch<double>::tau6(e64, phase, p->coef64, w64, 1, p->partials, p->div_blocks, d, s);
    launch_reduce(p->partials, p->div_blocks, 7, p->red, s);
    Launch<double>::zr2c(w64, S64, 6, d, t.tw[2], s);
    Launch<double>::yfft(S64, 6, d, t.tw[1], 0, s);
    launch_xeta6<double, T>(S64, d, t.tw[0], wt64, nullptr, p->op, XETA_STORE, static_cast<cpx<T>*>(p->dbase6), s);
    HIP_TRY(hipMemsetAsync(p->dlt, 0, 6 * (size_t)N * sizeof(T), s));
    HIP_TRY(hipMemcpyAsync(p->h_red, p->red, 7 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int i = 0; i < 6; ++i) mean_hi[i] = p->h_red[1 + i] / (double)N;
    it = static_cast<T*>(p->dlt);
    rf = static_cast<const T*>(p->rfield);
    anchored = true;
    ++refinements;
    return FE_OK;
  };

  // float64 re-anchor at the strain eps (+ it if anchored)
  auto reanchor = [&]() -> fe_status {
    if (!p->displacement) return reanchor6();
    const size_t spec = (size_t)spec_size(d);
    {
      fe_status ss = sync_iterate();
      if (ss != FE_OK) return ss;
    }
    if (!p->dlt) {
      HIP_TRY(dmalloc(p, &p->dlt_alt, 6 * (size_t)N * sizeof(T)));
      HIP_TRY(dmalloc(p, &p->dlt, 6 * (size_t)N * sizeof(T)));
      HIP_TRY(dmalloc(p, &p->rfield, 6 * (size_t)N * sizeof(T)));
      HIP_TRY(dmalloc(p, &p->dsig_hi, 3 * (size_t)N * sizeof(T)));
      HIP_TRY(dmalloc(p, (void**)&p->d64, 3 * (size_t)N * sizeof(double)));
      HIP_TRY(dmalloc(p, (void**)&p->s64, 3 * spec * sizeof(cpx<double>)));
    }
    if (anchored) Launch<T>::axpy(eps, it, 6 * N, s);
    const int nb = launch_div64<T>(eps, phase, p->coef64, p->d64, static_cast<T*>(p->dsig_hi), p->partials, d,
                                   p->op, s);
    launch_reduce(p->partials, nb, 7, p->red, s);
    const Tables<double>& t = p->t64;
    Launch<double>::zr2c(p->d64, p->s64, 3, d, t.tw[2], s);
    Launch<double>::yfft(p->s64, 3, d, t.tw[1], 0, s);
    Launch<double>::xgreen3(p->s64, d, t.tw[0], wave_tables<double>(p), g64, p->op, s);
    Launch<double>::yfft(p->s64, 3, d, t.tw[1], 1, s);
    Launch<double>::zc2r(p->s64, p->d64, 3, d, t.tw[2], s);
    launch_residual<T>(p->d64, eps, g64, static_cast<T*>(p->rfield), d, p->op, s);
    HIP_TRY(hipMemsetAsync(p->dlt, 0, 6 * (size_t)N * sizeof(T), s));
    HIP_TRY(hipMemcpyAsync(p->h_red, p->red, 7 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int i = 0; i < 6; ++i) mean_hi[i] = p->h_red[1 + i] / (double)N;
    it = static_cast<T*>(p->dlt);
    nxt = static_cast<T*>(p->dlt_alt);
    rf = static_cast<const T*>(p->rfield);
    dbase = static_cast<const T*>(p->dsig_hi);
    anchored = true;
    have_D = false;
    ++refinements;
    return FE_OK;
  };
  // float64 eta of the strain eps (+ it if anchored), folding it into eps
  // (folded: the correction is zero and eps holds the strain that was verified)
  bool folded = false;
  auto verify_total = [&](double* ev) -> fe_status {
    fe_status ss = sync_iterate();
    if (ss != FE_OK) return ss;
    if (anchored) {
      Launch<T>::axpy(eps, it, 6 * N, s);
      HIP_TRY(hipMemsetAsync(it, 0, 6 * (size_t)N * sizeof(T), s));
    }
    folded = true;
    return verify_fp64<T>(p, eps, phase, ev);
  };

  // without events (the allocation-free entry point) the loop is timed on the
  // host after a stream synchronisation and the convergence check is not
  // overlapped with the next iteration
  const auto host_t0 = std::chrono::steady_clock::now();
  if (p->ev0) HIP_TRY(hipEventRecord(p->ev0, s));
  PassTimer tm(p, p->opt.timing != 0);
  fe_status status = FE_NOT_CONVERGED;
  double eta = NAN, prev_eta = INFINITY, mean[6] = {0, 0, 0, 0, 0, 0};
  auto record = [&](int kk, double e) {
    if (kk >= out->history_capacity) return;
    if (out->eta_history) out->eta_history[kk] = e;
    if (out->mean_stress_history)
      for (int i = 0; i < 6; ++i) out->mean_stress_history[6 * kk + i] = mean[i];
  };
  double verified = NAN, last_verified = INFINITY;
  const int W = 10;
  std::vector<double> hist;
  int rising = 0, k = 0, last_anchor = 0;
  int anchor_gap = 2 * W;  // iterations between stagnation re-anchors; doubles after each (slow but steady runs)
  double best = INFINITY;  // float32 without re-anchoring: best eta and where it was reached
  int best_k = 0;
  bool need_anchor = false;
  for (k = 0;; ++k) {
    if (need_anchor) {
      fe_status rs = reanchor();
      if (rs != FE_OK) return rs;
      need_anchor = false;
      if (refinements > 1) anchor_gap = std::min(2 * anchor_gap, 200);
      last_anchor = k;
      rising = 0;
      prev_eta = INFINITY;
    }
    const bool check = (k % every == 0) || k == max_iter;
    if (p->displacement) {
      if (!have_D) {
        tm.run(FE_PASS_POINTWISE, [&] { nb_D = Launch<T>::div(it, phase, coef, R, dbase, p->partials, d, p->op, s); });
        have_D = true;
      }
      if (check) tm.run(FE_PASS_ETA, [&] { launch_reduce(p->partials, nb_D, 7, p->red, s); });
    } else if (check) {
      tm.run(FE_PASS_ETA, [&] {
        Launch<T>::tau6(it, phase, coef, R, 1, p->partials, p->div_blocks, d, s);
        launch_reduce(p->partials, p->div_blocks, 7, p->red, s);
        Launch<T>::zr2c(R, S, 6, d, tb.tw[2], s);
        Launch<T>::yfft(S, 6, d, tb.tw[1], 0, s);
        const int xblk = anchored ? launch_xeta6<T, T>(S, d, tb.tw[0], wt, p->partials2, p->op, XETA_BASE,
                                                       static_cast<cpx<T>*>(p->dbase6), s)
                                  : Launch<T>::xeta6(S, d, tb.tw[0], wt, p->partials2, p->op, s);
        launch_reduce(p->partials2, xblk, 1, p->red + 8, s);
      });
    }
    // Displacement form: the passes of iteration k are queued before eta^k is
    // read back, so the GPU works while the host decides.  They write only
    // nxt, R (the displacement), R2 and the partial sums, never it: when the
    // check stops, re-anchors or verifies (which may move it), the queued
    // iteration is dropped and the divergence of it is recomputed.
    bool queued = false, dropped = false;
    auto enqueue_passes = [&]() {
      tm.run(FE_PASS_ZFWD, [&] { Launch<T>::zr2c(R, S, 3, d, tb.tw[2], s); });
      tm.run(FE_PASS_YFWD, [&] { Launch<T>::yfft(S, 3, d, tb.tw[1], 0, s); });
      tm.run(FE_PASS_XGREEN, [&] { Launch<T>::xgreen3(S, d, tb.tw[0], wt, g, p->op, s); });
      tm.run(FE_PASS_YINV, [&] { Launch<T>::yfft(S, 3, d, tb.tw[1], 1, s); });
      tm.run(FE_PASS_ZINV, [&] { Launch<T>::zc2r(S, R, 3, d, tb.tw[2], s); });
      // eps^(k+1) (into nxt) and the divergence of its tau (into R2) with eta's sums
      tm.run(FE_PASS_UPDATE, [&] {
        nb_D = Launch<T>::update_div(R, it, nxt, phase, coef, g, rf, R2, dbase, p->partials, d, p->op, accel, s);
      });
    };
    // Queue ahead only while this check is unlikely to end the run: when the
    // eta just read may reach tol (the last ratio extrapolated once, with a
    // factor 3 of margin) the queued iteration would be dropped, costing a
    // whole iteration instead of the host round trip it hides.
    bool ahead = p->displacement && k < max_iter && p->evc;
    if (ahead && !hist.empty()) {
      const size_t nh = hist.size();
      const double r = nh >= 2 && hist[nh - 2] > 0.0 ? hist[nh - 1] / hist[nh - 2] : 1.0;
      if (hist[nh - 1] * std::min(r, 1.0) <= 3.0 * tol) ahead = false;
    }
    if (check) {
      HIP_TRY(hipMemcpyAsync(p->h_red, p->red, 9 * sizeof(double), hipMemcpyDeviceToHost, s));
      if (ahead) {
        HIP_TRY(hipEventRecord(p->evc, s));
        enqueue_passes();
        queued = true;
        HIP_TRY(hipEventSynchronize(p->evc));
      } else {
        HIP_TRY(hipStreamSynchronize(s));
      }
      for (int i = 0; i < 6; ++i) mean[i] = mean_hi[i] + p->h_red[1 + i] / (double)N;
      const double nrm = frob(mean);
      eta = p->displacement ? std::sqrt(p->h_red[0] / (double)N) / nrm : std::sqrt(p->h_red[8]) / ((double)N * nrm);
      record(k, eta);
      hist.push_back(eta);
      if (!std::isfinite(eta)) {
        status = FE_DIVERGED;
        break;
      }
      if (eta <= tol) {
        if (!can_refine) {
          status = FE_OK;
          break;
        }
        // the float32 measure says converged: confirm in float64
        dropped = true;
        fe_status vs = verify_total(&verified);
        if (vs != FE_OK) return vs;
        if (verified <= tol) {
          status = FE_OK;
          break;
        }
        // not there in float64.  If the previous float64 check was no worse,
        // the float32-stored strain cannot get closer (storage floor): stop.
        if (verified > 0.9 * last_verified) {
          status = FE_NOT_CONVERGED;
          break;
        }
        last_verified = verified;
        // re-anchor at this strain and redo this iteration from the new anchor
        // (at most once per anchor)
        if (k > last_anchor || !anchored) {
          need_anchor = true;
          --k;
          continue;
        }
      }
      if (k >= max_iter) {
        status = FE_NOT_CONVERGED;
        break;
      }
      rising = eta > prev_eta ? rising + 1 : 0;
      prev_eta = eta;
      if (p->opt.diverge_window > 0 && rising >= p->opt.diverge_window && !can_refine) {
        status = FE_DIVERGED;
        break;
      }
      // stagnation of the float32 iteration: less than 30% decrease over W checks
      const int nh = (int)hist.size();
      if (can_refine && !need_anchor && k - last_anchor >= anchor_gap && nh > W && eta > 0.7 * hist[nh - 1 - W])
        need_anchor = true;
      // the float32 floor after fast convergence: the last 2 checks gained less
      // than 30% where the 5 before fell by at least 0.8x per check
      if (can_refine && !need_anchor && k - last_anchor >= 8 && nh >= 8 && eta > 0.7 * hist[nh - 3] &&
          hist[nh - 3] < std::pow(0.8, 5) * hist[nh - 8])
        need_anchor = true;
      // its first sign in a steady geometric decrease: the last ratio exceeds
      // 1.3x the mean of the 4 ratios before the previous one, which stayed
      // below 0.8 and within 1.3x of each other (the float32 error adds to
      // eta in quadrature, so the ratio rises over a few checks before eta
      // stalls; the previous ratio may already be rising)
      if (can_refine && !need_anchor && k - last_anchor >= 8 && nh >= 7 && eta < 1e-3 * hist[0]) {
        double rmin = INFINITY, rmax = 0.0, lsum = 0.0;
        for (int i = nh - 6; i < nh - 2; ++i) {
          const double r = hist[i] / hist[i - 1];
          rmin = std::fmin(rmin, r);
          rmax = std::fmax(rmax, r);
          lsum += std::log(r);
        }
        if (rmax < 0.8 && rmax < 1.3 * rmin && hist[nh - 1] > 1.3 * std::exp(0.25 * lsum) * hist[nh - 2])
          need_anchor = true;
      }
      // float32 without re-anchoring: stop at the storage floor (no 5% gain in 100 iterations)
      if (!can_refine && sizeof(T) == 4) {
        if (eta < 0.95 * best) {
          best = eta;
          best_k = k;
        } else if (k - best_k >= 100) {
          status = FE_NOT_CONVERGED;
          break;
        }
      }
      if (can_refine && p->opt.diverge_window > 0 && rising >= p->opt.diverge_window && refinements > 3) {
        status = FE_DIVERGED;
        break;
      }
    }
    if (p->displacement) {
      if (!queued && !dropped) enqueue_passes();
      if (dropped) {
        have_D = false;  // R holds a displacement now; the divergence of it is recomputed
      } else {
        std::swap(it, nxt);
        std::swap(R, R2);
        have_D = true;
      }
    } else {
      tm.run(FE_PASS_POINTWISE, [&] { Launch<T>::tau6(it, phase, coef, R, 0, nullptr, p->div_blocks, d, s); });
      tm.run(FE_PASS_ZFWD, [&] { Launch<T>::zr2c(R, S, 6, d, tb.tw[2], s); });
      tm.run(FE_PASS_YFWD, [&] { Launch<T>::yfft(S, 6, d, tb.tw[1], 0, s); });
      tm.run(FE_PASS_XGREEN, [&] { Launch<T>::xgreen6(S, d, tb.tw[0], wt, anchored ? gz : g, p->op, s); });
      tm.run(FE_PASS_YINV, [&] { Launch<T>::yfft(S, 6, d, tb.tw[1], 1, s); });
      tm.run(FE_PASS_ZINV, [&] { Launch<T>::zc2r(S, R, 6, d, tb.tw[2], s); });
      tm.run(FE_PASS_UPDATE, [&] { Launch<T>::update6(R, it, phase, coef, d, accel, s, anchored ? rf : nullptr); });
    }
    HIP_TRY(hipGetLastError());
  }
  const bool verified_final = folded && status == FE_OK;  // eps is the strain just verified
  if (anchored && !verified_final) {  // the returned strain is anchor + correction
    Launch<T>::axpy(eps, it, 6 * N, s);
    HIP_TRY(hipMemsetAsync(it, 0, 6 * (size_t)N * sizeof(T), s));
  } else {
    fe_status ss = sync_iterate();
    if (ss != FE_OK) return ss;
  }
  float ms_elapsed = 0.f;
  if (p->ev1) {
    HIP_TRY(hipEventRecord(p->ev1, s));
    HIP_TRY(hipEventSynchronize(p->ev1));
    tm.flush();
    HIP_TRY(hipEventElapsedTime(&ms_elapsed, p->ev0, p->ev1));
  } else {
    HIP_TRY(hipStreamSynchronize(s));
    ms_elapsed = (float)(std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - host_t0).count());
  }
  HIP_TRY(hipGetLastError());
  for (int i = 0; i < 8; ++i) {
    out->pass_seconds[i] = tm.sec[i];
    out->pass_launches[i] = tm.launches[i];
  }
  out->refinements = refinements;

  if (out->stress) Launch<T>::stress(eps, phase, coef, static_cast<T*>(out->stress), N, s);
  double ev = eta;
  if (sizeof(T) == 4) {
    if (verified_final) {
      ev = verified;
    } else {
      fe_status vs = verify_fp64<T>(p, eps, phase, &ev);
      if (vs != FE_OK) return vs;
    }
  }
  HIP_TRY(hipStreamSynchronize(s));
  out->iterations = k;
  out->eta = eta;
  out->eta_verify_fp64 = ev;
  out->seconds = ms_elapsed * 1e-3;
  for (int i = 0; i < 6; ++i) out->mean_stress[i] = mean[i];
  if (status == FE_NOT_CONVERGED)
    fail(status, "not converged after %d iterations (eta = %.3e, tol = %.3e)", k, eta, tol);
  else if (status == FE_DIVERGED)
    fail(status, "diverged at iteration %d (eta = %.3e)", k, eta);
  return status;
}

extern "C" fe_status fe_solve(fe_plan* p, const uint8_t* phase, fe_materials materials, const double macro_strain[6],
                              double tol, const void* strain_init, fe_result* out) {
  if (!p) return fail(FE_ERR_INVALID_ARG, "plan is NULL");
  if (!phase) return fail(FE_ERR_INVALID_ARG, "phase is NULL");
  if (!macro_strain) return fail(FE_ERR_INVALID_ARG, "macro_strain is NULL");
  if (!out) return fail(FE_ERR_INVALID_ARG, "out is NULL");
  if (!(tol > 0.0) || !std::isfinite(tol)) return fail(FE_ERR_INVALID_ARG, "tol must be finite and > 0");
  for (int i = 0; i < 6; ++i)
    if (!std::isfinite(macro_strain[i])) return fail(FE_ERR_INVALID_ARG, "macro_strain[%d] is not finite", i);
  if (out->history_capacity < 0) return fail(FE_ERR_INVALID_ARG, "history_capacity < 0");
  if (out->history_capacity > 0 && !out->eta_history && !out->mean_stress_history)
    return fail(FE_ERR_INVALID_ARG, "eta_history and mean_stress_history are NULL with a positive capacity");
  fe_status st = validate_materials(materials);
  if (st != FE_OK) return st;
  if (p->scheme == FE_CONJUGATE_GRADIENT && strain_init)
    return fail(FE_ERR_UNSUPPORTED, "conjugate gradients start from the applied strain (strain_init must be NULL)");
  HIP_TRY(hipSetDevice(p->device));
  if (p->opt.precision == FE_FP64)
    return solve_impl<double>(p, phase, materials, macro_strain, tol, strain_init, out);
  return solve_impl<float>(p, phase, materials, macro_strain, tol, strain_init, out);
}

// ---------------------------------------------------------------------------
// allocation-free solve: the workspace lives in a static device array
// ---------------------------------------------------------------------------
// Every device the library runs on holds its own copy of this array until the
// process ends.  Host code never passes its name to a kernel or a copy: the
// name is a host-side stand-in, the device address comes from
// hipGetSymbolAddress, taken once per device with that device current.
static __device__ __align__(256) unsigned char scratch[FE_STATIC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[kMaxDevices] = {};

fe_status scratch_address(int dev, unsigned char** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(FE_ERR_UNSUPPORTED, "device index %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(FE_ERR_DEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<unsigned char*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return FE_OK;
}

// Carve the plan's buffers out of [base, base + cap) (nullptr base: count
// only); returns the bytes needed.
template <typename T>
size_t carve_static(fe_plan* p, unsigned char* base, size_t cap, std::vector<std::vector<T>>* host_tables) {
  size_t used = 0;
  bool fits = true;
  auto take = [&](size_t bytes) -> void* {
    const size_t off = (used + 255) & ~(size_t)255;
    used = off + bytes;
    if (used > cap) fits = false;
    return base && fits ? base + off : nullptr;
  };
  const Dims d = p->d;
  const long long N = d.N;
  const size_t spec = (size_t)spec_size(d);
  const size_t lines = (size_t)d.Hp * p->grid.ny;
  p->R = take(3 * (size_t)N * sizeof(T));
  p->R2 = take(3 * (size_t)N * sizeof(T));
  p->eps_alt = take(6 * (size_t)N * sizeof(T));
  p->S = take(3 * spec * 2 * sizeof(T));
  p->partials = static_cast<double*>(take(p->partial_count * sizeof(double)));
  p->partials2 = static_cast<double*>(take((lines + 1) * sizeof(double)));
  p->red = static_cast<double*>(take(16 * sizeof(double)));
  p->flag = static_cast<int*>(take(sizeof(int)));
  p->coef = take(256 * sizeof(PhaseCoef<double>));
  p->coef64 = static_cast<PhaseCoef<double>*>(take(256 * sizeof(PhaseCoef<double>)));
  Tables<T>& t = tables_mut<T>(p);
  const int n[3] = {p->grid.nx, p->grid.ny, p->grid.nz};
  for (int a = 0; a < 3; ++a) {
    t.tw[a] = static_cast<cpx<T>*>(take(2 * (size_t)n[a] * sizeof(T)));
    t.wave[a] = static_cast<T*>(take(2 * (size_t)n[a] * sizeof(T)));
    if (host_tables) {
      std::vector<double> tw = twiddles(n[a]), wv = wave_table(n[a], p->op);
      host_tables->emplace_back(tw.begin(), tw.end());
      host_tables->emplace_back(wv.begin(), wv.end());
    }
  }
  return used;
}
}  // namespace

extern "C" fe_status fe_solve_static(fe_grid g, fe_discretization disc, fe_scheme scheme, const fe_plan_options* opt,
                                     const uint8_t* phase, fe_materials materials, const double macro_strain[6],
                                     double tol, const void* strain_init, fe_result* out) {
  fe_plan_options o;
  fe_plan_options_default(&o);
  if (opt) {
    if (opt->struct_size != sizeof(fe_plan_options))
      return fail(FE_ERR_INVALID_ARG, "fe_plan_options.struct_size is %u, expected %zu", opt->struct_size,
                  sizeof(fe_plan_options));
    o = *opt;
  }
  if (disc != FE_GREEN_WP && disc != FE_GREEN_ROT)
    return fail(disc >= FE_GREEN_MS && disc <= FE_GREEN_MS_SYMMETRIZED ? FE_ERR_UNSUPPORTED : FE_ERR_INVALID_ARG,
                "fe_solve_static runs the WP and ROT operators");
  if (scheme != FE_DIRECT && scheme != FE_ACCELERATED)
    return fail(scheme == FE_CONJUGATE_GRADIENT ? FE_ERR_UNSUPPORTED : FE_ERR_INVALID_ARG,
                "fe_solve_static runs the direct and accelerated schemes");
  if (o.precision != FE_FP32 && o.precision != FE_FP64)
    return fail(FE_ERR_INVALID_ARG, "unknown precision %d", (int)o.precision);
  if (o.timing) return fail(FE_ERR_UNSUPPORTED, "fe_solve_static does not time passes (timing must be 0)");
  if (o.max_iter < 0 || o.check_every < 1 || o.diverge_window < 0)
    return fail(FE_ERR_INVALID_ARG, "max_iter, check_every or diverge_window out of range");
  if (o.ref_rule != FE_REF_PAPER && o.ref_rule != FE_REF_EXPLICIT)
    return fail(FE_ERR_INVALID_ARG, "unknown ref_rule %d", o.ref_rule);
  if (o.ref_rule == FE_REF_PAPER && scheme == FE_DIRECT && !(o.ds_beta > 0.0 && std::isfinite(o.ds_beta)))
    return fail(FE_ERR_INVALID_ARG, "ds_beta must be positive and finite");
  if (o.ref_rule == FE_REF_EXPLICIT &&
      !(std::isfinite(o.E0) && o.E0 > 0.0 && std::isfinite(o.nu0) && o.nu0 > -1.0 && o.nu0 < 0.5))
    return fail(FE_ERR_INVALID_ARG, "explicit reference needs E0 > 0 and -1 < nu0 < 0.5");
  const int n[3] = {g.nx, g.ny, g.nz};
  for (int a = 0; a < 3; ++a) {
    if (n[a] <= 0) return fail(FE_ERR_INVALID_ARG, "grid dimension %d is %d", a, n[a]);
    if (!(a == 2 ? supported_z_length(n[a]) : supported_length(n[a])))
      return fail(FE_ERR_UNSUPPORTED, "grid dimension %d = %d: need 2^a or 3*2^a in [4, 1024] (nz: or 1)", a, n[a]);
  }
  if (!phase || !macro_strain || !out) return fail(FE_ERR_INVALID_ARG, "phase, macro_strain or out is NULL");
  if (!out->strain) return fail(FE_ERR_INVALID_ARG, "fe_solve_static needs out->strain (it keeps no iterate)");
  if (!(tol > 0.0) || !std::isfinite(tol)) return fail(FE_ERR_INVALID_ARG, "tol must be finite and > 0");
  for (int i = 0; i < 6; ++i)
    if (!std::isfinite(macro_strain[i])) return fail(FE_ERR_INVALID_ARG, "macro_strain[%d] is not finite", i);
  if (out->history_capacity < 0) return fail(FE_ERR_INVALID_ARG, "history_capacity < 0");
  if (out->history_capacity > 0 && !out->eta_history && !out->mean_stress_history)
    return fail(FE_ERR_INVALID_ARG, "eta_history and mean_stress_history are NULL with a positive capacity");
  fe_status st = validate_materials(materials);
  if (st != FE_OK) return st;

  fe_plan p;  // no allocation: every buffer is a slice of the static array, no events
  p.grid = g;
  p.disc = disc;
  p.scheme = scheme;
  p.opt = o;
  p.opt.refine = 0;  // float32 runs iterate in float32 only (re-anchoring needs more workspace)
  p.stream = (hipStream_t)o.hip_stream;
  p.op = disc == FE_GREEN_WP ? OP_WP : OP_ROT;
  p.displacement = true;
  p.d = make_dims(g.nx, g.ny, g.nz);
  const long long db = (p.d.N + kThreads - 1) / kThreads;
  p.div_blocks = (int)(db > kMaxReduceBlocks ? kMaxReduceBlocks : db);
  p.partial_count = (size_t)kMaxReduceBlocks * 7;
  const bool f64 = o.precision == FE_FP64;
  const size_t need = f64 ? carve_static<double>(&p, nullptr, SIZE_MAX, nullptr)
                          : carve_static<float>(&p, nullptr, SIZE_MAX, nullptr);
  if (need > (size_t)FE_STATIC_SCRATCH_BYTES)
    return fail(FE_ERR_UNSUPPORTED, "grid %dx%dx%d needs %zu bytes of workspace; the static scratch holds %zu",
                g.nx, g.ny, g.nz, need, (size_t)FE_STATIC_SCRATCH_BYTES);
  HIP_TRY(hipGetDevice(&p.device));
  unsigned char* base = nullptr;
  st = scratch_address(p.device, &base);
  if (st != FE_OK) return st;
  double h_red[16];
  p.h_red = h_red;
  std::vector<std::vector<double>> h64;
  std::vector<std::vector<float>> h32;
  if (f64)
    carve_static<double>(&p, base, FE_STATIC_SCRATCH_BYTES, &h64);
  else
    carve_static<float>(&p, base, FE_STATIC_SCRATCH_BYTES, &h32);
  for (int a = 0; a < 3; ++a) {
    if (f64) {
      HIP_TRY(hipMemcpyAsync(p.t64.tw[a], h64[2 * a].data(), h64[2 * a].size() * 8, hipMemcpyHostToDevice, p.stream));
      HIP_TRY(hipMemcpyAsync(p.t64.wave[a], h64[2 * a + 1].data(), h64[2 * a + 1].size() * 8, hipMemcpyHostToDevice,
                             p.stream));
    } else {
      HIP_TRY(hipMemcpyAsync(p.t32.tw[a], h32[2 * a].data(), h32[2 * a].size() * 4, hipMemcpyHostToDevice, p.stream));
      HIP_TRY(hipMemcpyAsync(p.t32.wave[a], h32[2 * a + 1].data(), h32[2 * a + 1].size() * 4, hipMemcpyHostToDevice,
                             p.stream));
    }
  }
  st = f64 ? solve_impl<double>(&p, phase, materials, macro_strain, tol, strain_init, out)
           : solve_impl<float>(&p, phase, materials, macro_strain, tol, strain_init, out);
  (void)hipStreamSynchronize(p.stream);  // the host tables and h_red outlive every queued copy
  return st;
}

extern "C" fe_status fe_effective_stiffness(fe_plan* p, const uint8_t* phase, fe_materials materials, double tol,
                                            double C_voigt[36], int32_t iterations[6]) {
  if (!C_voigt) return fail(FE_ERR_INVALID_ARG, "C_voigt is NULL");
  fe_status worst = FE_OK;
  for (int J = 0; J < 6; ++J) {
    double e[6] = {0, 0, 0, 0, 0, 0};
    e[J] = 1.0;
    fe_result r;
    std::memset(&r, 0, sizeof r);
    fe_status st = fe_solve(p, phase, materials, e, tol, nullptr, &r);
    if (st < 0) return st;
    if (st > worst) worst = st;
    for (int I = 0; I < 6; ++I) C_voigt[6 * I + J] = J < 3 ? r.mean_stress[I] : 0.5 * r.mean_stress[I];
    if (iterations) iterations[J] = r.iterations;
  }
  return worst;
}

extern "C" const char* fe_status_string(fe_status s) {
  switch (s) {
    case FE_OK: return "FE_OK";
    case FE_NOT_CONVERGED: return "FE_NOT_CONVERGED";
    case FE_DIVERGED: return "FE_DIVERGED";
    case FE_ERR_INVALID_ARG: return "FE_ERR_INVALID_ARG";
    case FE_ERR_UNSUPPORTED: return "FE_ERR_UNSUPPORTED";
    case FE_ERR_OOM: return "FE_ERR_OOM";
    case FE_ERR_DEVICE: return "FE_ERR_DEVICE";
  }
  return "FE_UNKNOWN_STATUS";
}

extern "C" const char* fe_last_error(void) { return last_error_text().c_str(); }

// ---------------------------------------------------------------------------
// batched solves
// ---------------------------------------------------------------------------
namespace {

template <typename T>
struct BatchClass {
  Dims d;
  std::vector<int> ids;  // sample indices of the batch in this class
  int ncoef = 1;
  int div_blocks = 0;
  T* eps = nullptr;   // returned strains (every retired sample's final iterate ends here)
  T* eps2 = nullptr;  // second iterate buffer of the fused update
  T* R = nullptr;
  T* R2 = nullptr;
  T* cur = nullptr;   // current iterate buffer (eps or eps2)
  T* nxt = nullptr;
  cpx<T>* S = nullptr;
  uint8_t* phase = nullptr;
  double* partials = nullptr;
  double* red = nullptr;
  PhaseCoef<T>* coef = nullptr;
  PhaseCoef<double>* coef64 = nullptr;
  GreenConst<T>* gcon = nullptr;
  int* active = nullptr;
  int* all = nullptr;
  cpx<T>* tw[3] = {nullptr, nullptr, nullptr};
  T* wave[3] = {nullptr, nullptr, nullptr};
  std::vector<int> act;  // host copy of the active list
  std::vector<int> rising;
  std::vector<double> prev;
  std::vector<double> best;
  std::vector<int> best_k;
  void release() {
    void* b[] = {eps, eps2, R, R2, S, phase, partials, red, coef, coef64, gcon, active, all, tw[0], tw[1], tw[2],
                 wave[0], wave[1], wave[2]};
    for (void* x : b)
      if (x) (void)hipFree(x);
  }
};

constexpr int kStallWindow = 100;

template <typename T>
fe_status alloc_class(BatchClass<T>& c, int op) {
  const size_t n = c.ids.size();
  const long long N = c.d.N;
  const size_t spec = (size_t)spec_size(c.d);
  HIP_TRY(hipMalloc((void**)&c.eps, n * 6 * N * sizeof(T)));
  HIP_TRY(hipMalloc((void**)&c.eps2, n * 6 * N * sizeof(T)));
  HIP_TRY(hipMalloc((void**)&c.R, n * 3 * N * sizeof(T)));
  HIP_TRY(hipMalloc((void**)&c.R2, n * 3 * N * sizeof(T)));
  c.cur = c.eps;
  c.nxt = c.eps2;
  HIP_TRY(hipMalloc((void**)&c.S, n * 3 * spec * sizeof(cpx<T>)));
  HIP_TRY(hipMalloc((void**)&c.phase, n * N));
  HIP_TRY(hipMalloc((void**)&c.partials, n * (size_t)c.div_blocks * 7 * sizeof(double)));
  HIP_TRY(hipMalloc((void**)&c.red, n * 8 * sizeof(double)));
  HIP_TRY(hipMalloc((void**)&c.coef, n * c.ncoef * sizeof(PhaseCoef<T>)));
  HIP_TRY(hipMalloc((void**)&c.coef64, n * c.ncoef * sizeof(PhaseCoef<double>)));
  HIP_TRY(hipMalloc((void**)&c.gcon, n * sizeof(GreenConst<T>)));
  HIP_TRY(hipMalloc((void**)&c.active, n * sizeof(int)));
  HIP_TRY(hipMalloc((void**)&c.all, n * sizeof(int)));
  const int dims[3] = {c.d.nx, c.d.ny, c.d.nz};
  for (int a = 0; a < 3; ++a) {
    std::vector<double> tw = twiddles(dims[a]), wv = wave_table(dims[a], op);
    std::vector<T> twt(tw.begin(), tw.end()), wvt(wv.begin(), wv.end());
    HIP_TRY(hipMalloc((void**)&c.tw[a], twt.size() * sizeof(T)));
    HIP_TRY(hipMalloc((void**)&c.wave[a], wvt.size() * sizeof(T)));
    HIP_TRY(hipMemcpy(c.tw[a], twt.data(), twt.size() * sizeof(T), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c.wave[a], wvt.data(), wvt.size() * sizeof(T), hipMemcpyHostToDevice));
  }
  return FE_OK;
}

template <typename T>
fe_status solve_batched_impl(int op, bool accel, const fe_plan_options& o, const fe_batch_desc* desc, double tol,
                             fe_batch_result* results, double* seconds, const float* const* init = nullptr) {
  hipStream_t s = (hipStream_t)o.hip_stream;
  const int ns = desc->n_samples;
  // group samples by grid
  std::vector<BatchClass<T>> cls;
  for (int i = 0; i < ns; ++i) {
    const fe_grid& g = desc->grids[i];
    size_t c = 0;
    for (; c < cls.size(); ++c)
      if (cls[c].d.nx == g.nx && cls[c].d.ny == g.ny && cls[c].d.nz == g.nz) break;
    if (c == cls.size()) {
      BatchClass<T> bc;
      bc.d = make_dims(g.nx, g.ny, g.nz);
      cls.push_back(bc);
    }
    cls[c].ids.push_back(i);
    cls[c].ncoef = std::max(cls[c].ncoef, desc->materials[i].n_phases);
  }
  struct Guard {
    std::vector<BatchClass<T>>& v;
    ~Guard() {
      for (auto& c : v) c.release();
    }
  } guard{cls};

  int* hflag = nullptr;
  HIP_TRY(hipMalloc((void**)&hflag, sizeof(int)));
  struct FlagGuard {
    int* f;
    ~FlagGuard() { (void)hipFree(f); }
  } fg{hflag};
  HIP_TRY(hipMemsetAsync(hflag, 0, sizeof(int), s));

  for (auto& c : cls) {
    const long long N = c.d.N;
    c.div_blocks = div_partial_count(c.d);
    fe_status st = alloc_class(c, op);
    if (st != FE_OK) return st;
    const size_t n = c.ids.size();
    std::vector<PhaseCoef<T>> cT(n * c.ncoef);
    std::vector<PhaseCoef<double>> c64(n * c.ncoef);
    std::vector<GreenConst<T>> gv(n);
    std::vector<int> idx(n);
    for (size_t j = 0; j < n; ++j) {
      const int i = c.ids[j];
      idx[j] = (int)j;
      const fe_materials& m = desc->materials[i];
      const RefMedium ref = reference_medium(o, accel ? FE_ACCELERATED : FE_DIRECT, m);
      std::vector<PhaseCoef<double>> pc = phase_coefs(m, ref);
      for (int q = 0; q < m.n_phases; ++q) {
        c64[j * c.ncoef + q] = pc[q];
        PhaseCoef<T>& t = cT[j * c.ncoef + q];
        t.lam = T(pc[q].lam);
        t.mu = T(pc[q].mu);
        t.dlam = T(pc[q].dlam);
        t.dmu = T(pc[q].dmu);
        t.ak = T(pc[q].ak);
        t.am = T(pc[q].am);
        t.pad0 = t.pad1 = T(0);
      }
      GreenConst<T>& g = gv[j];
      g.lam0 = T(ref.lam0);
      g.mu0 = T(ref.mu0);
      g.cr = T((ref.lam0 + ref.mu0) / (ref.lam0 + 2.0 * ref.mu0));
      g.s1 = T(1.0 / (2.0 * ref.mu0));
      g.s2 = T(ref.lam0 / (2.0 * ref.mu0 * (3.0 * ref.lam0 + 2.0 * ref.mu0)));
      g.inv_n = T(1.0 / (double)N);
      for (int q = 0; q < 6; ++q) g.macro[q] = T(desc->macro_strain[6 * i + q]);
      HIP_TRY(hipMemcpyAsync(c.phase + j * N, desc->phase[i], N, hipMemcpyDeviceToDevice, s));
      Launch<T>::check_phase(c.phase + j * N, N, m.n_phases, hflag, s);
      if (init && init[i])  // a float32 start (the persistent solve's iterate)
        Launch<T>::convert_to(c.eps + j * 6 * N, init[i], 0, 6 * N, s);
      else
        Launch<T>::fill_macro(c.eps + j * 6 * N, N, desc->macro_strain + 6 * i, s);
    }
    HIP_TRY(hipMemcpyAsync(c.coef, cT.data(), cT.size() * sizeof(PhaseCoef<T>), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(c.coef64, c64.data(), c64.size() * sizeof(PhaseCoef<double>), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(c.gcon, gv.data(), n * sizeof(GreenConst<T>), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(c.all, idx.data(), n * sizeof(int), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(c.active, idx.data(), n * sizeof(int), hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    c.act = idx;
    c.rising.assign(n, 0);
    c.prev.assign(n, INFINITY);
    c.best.assign(n, INFINITY);
    c.best_k.assign(n, 0);
  }
  int flag = 0;
  HIP_TRY(hipMemcpy(&flag, hflag, sizeof(int), hipMemcpyDeviceToHost));
  if (flag) return fail(FE_ERR_INVALID_ARG, "a phase map holds a label >= its n_phases");

  for (int i = 0; i < ns; ++i) {
    results[i].status = FE_NOT_CONVERGED;
    results[i].iterations = 0;
  }
  // one stream per grid class (default priority): the classes are
  // independent, so their launches overlap and small grids fill the chip
  // together; every iteration joins them on the host
  struct Streams {
    std::vector<hipStream_t> v;
    std::vector<hipEvent_t> ev;
    ~Streams() {
      for (hipStream_t q : v) (void)hipStreamDestroy(q);
      for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }
  } cs;
  for (size_t c = 0; c < cls.size(); ++c) {
    hipStream_t q = nullptr;
    HIP_TRY(hipStreamCreateWithFlags(&q, hipStreamNonBlocking));
    cs.v.push_back(q);
    hipEvent_t e = nullptr;
    HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    cs.ev.push_back(e);
  }
  auto join = [&]() -> fe_status {
    for (hipStream_t q : cs.v) HIP_TRY(hipStreamSynchronize(q));
    return FE_OK;
  };
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  HIP_TRY(hipEventRecord(e0, s));
  for (hipStream_t q : cs.v) HIP_TRY(hipStreamWaitEvent(q, e0, 0));
  std::vector<double> hred;
  // eta^0: divergence of eps_bar for every sample
  for (size_t ci = 0; ci < cls.size(); ++ci) {
    auto& c = cls[ci];
    hipStream_t s = cs.v[ci];
    const int na = (int)c.act.size();
    const Batch bt{c.active, c.ncoef};
    const int nb = Launch<T>::div(c.cur, c.phase, c.coef, c.R, nullptr, c.partials, c.d, op, s, bt, na);
    launch_reduce(c.partials, nb, 7, c.red, s, c.active, na);
  }
  for (int k = 0;; ++k) {
    {
      fe_status js = join();
      if (js != FE_OK) return js;
    }
    bool left = false;
    for (size_t ci = 0; ci < cls.size(); ++ci) {
      auto& c = cls[ci];
      hipStream_t s = cs.v[ci];
      if (c.act.empty()) continue;
      hred.resize(c.ids.size() * 8);
      HIP_TRY(hipMemcpy(hred.data(), c.red, hred.size() * sizeof(double), hipMemcpyDeviceToHost));
      std::vector<int> keep;
      for (int j : c.act) {
        const double* r = &hred[8 * j];
        double mean[6];
        for (int q = 0; q < 6; ++q) mean[q] = r[1 + q] / (double)c.d.N;
        const double eta = std::sqrt(r[0] / (double)c.d.N) / frob(mean);
        fe_batch_result& out = results[c.ids[j]];
        out.iterations = k;
        out.eta = eta;
        for (int q = 0; q < 6; ++q) out.mean_stress[q] = mean[q];
        bool done = true;
        // same stopping order as the single-sample solve with refinement off
        if (!std::isfinite(eta)) {
          out.status = FE_DIVERGED;
        } else if (eta <= tol) {
          out.status = FE_OK;
        } else if (k >= o.max_iter) {
          out.status = FE_NOT_CONVERGED;
        } else {
          c.rising[j] = eta > c.prev[j] ? c.rising[j] + 1 : 0;
          c.prev[j] = eta;
          if (o.diverge_window > 0 && c.rising[j] >= o.diverge_window) {
            out.status = FE_DIVERGED;
          } else if (eta < 0.95 * c.best[j]) {  // storage floor: no 5% gain over kStallWindow iterations
            c.best[j] = eta;
            c.best_k[j] = k;
            done = false;
          } else if (k - c.best_k[j] >= kStallWindow) {
            out.status = FE_NOT_CONVERGED;
          } else {
            done = false;
          }
        }
        if (!done) {
          keep.push_back(j);
        } else if (c.cur != c.eps) {  // the final iterate goes to the returned buffer
          HIP_TRY(hipMemcpyAsync(c.eps + (size_t)j * 6 * c.d.N, c.cur + (size_t)j * 6 * c.d.N,
                                 6 * c.d.N * sizeof(T), hipMemcpyDeviceToDevice, s));
        }
      }
      c.act.swap(keep);  // c.act stays untouched until the next synchronisation
      if (!c.act.empty()) {
        left = true;
        HIP_TRY(hipMemcpyAsync(c.active, c.act.data(), c.act.size() * sizeof(int), hipMemcpyHostToDevice, s));
      }
    }
    if (!left) break;
    for (size_t ci = 0; ci < cls.size(); ++ci) {
      auto& c = cls[ci];
      hipStream_t s = cs.v[ci];
      const int na = (int)c.act.size();
      if (!na) continue;
      const Batch bt{c.active, c.ncoef};
      const WaveTables<T> wt{c.wave[0], c.wave[1], c.wave[2]};
      GreenConst<T> g0;
      std::memset(&g0, 0, sizeof g0);
      Launch<T>::zr2c(c.R, c.S, 3, c.d, c.tw[2], s, bt, na);
      Launch<T>::yfft(c.S, 3, c.d, c.tw[1], 0, s, bt, na);
      Launch<T>::xgreen3(c.S, c.d, c.tw[0], wt, g0, op, s, bt, c.gcon, na);
      Launch<T>::yfft(c.S, 3, c.d, c.tw[1], 1, s, bt, na);
      Launch<T>::zc2r(c.S, c.R, 3, c.d, c.tw[2], s, bt, na);
      const int nb = Launch<T>::update_div(c.R, c.cur, c.nxt, c.phase, c.coef, g0, nullptr, c.R2, nullptr, c.partials,
                                           c.d, op, accel, s, bt, c.gcon, na);
      launch_reduce(c.partials, nb, 7, c.red, s, c.active, na);
      std::swap(c.cur, c.nxt);
      std::swap(c.R, c.R2);
    }
    HIP_TRY(hipGetLastError());
  }
  for (size_t ci = 0; ci < cls.size(); ++ci) {  // the caller's stream after every class
    HIP_TRY(hipEventRecord(cs.ev[ci], cs.v[ci]));
    HIP_TRY(hipStreamWaitEvent(s, cs.ev[ci], 0));
  }
  HIP_TRY(hipEventRecord(e1, s));
  HIP_TRY(hipEventSynchronize(e1));
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (seconds) *seconds = ms * 1e-3;

  // float64 verification and outputs
  for (auto& c : cls) {
    const int n = (int)c.ids.size();
    const Batch bt{c.all, c.ncoef};
    const int nb = launch_div64<T>(c.eps, c.phase, c.coef64, nullptr, nullptr, c.partials, c.d, op, s, bt, n);
    launch_reduce(c.partials, nb, 7, c.red, s, c.all, n);
    hred.resize((size_t)n * 8);
    HIP_TRY(hipMemcpyAsync(hred.data(), c.red, hred.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int j = 0; j < n; ++j) {
      const double* r = &hred[8 * j];
      double mean[6];
      for (int q = 0; q < 6; ++q) mean[q] = r[1 + q] / (double)c.d.N;
      results[c.ids[j]].eta_verify_fp64 = std::sqrt(r[0] / (double)c.d.N) / frob(mean);
      if (desc->strain && desc->strain[c.ids[j]])
        HIP_TRY(hipMemcpyAsync(desc->strain[c.ids[j]], c.eps + (size_t)j * 6 * c.d.N, 6 * c.d.N * sizeof(T),
                               hipMemcpyDeviceToDevice, s));
    }
  }
  HIP_TRY(hipStreamSynchronize(s));
  fe_status worst = FE_OK;
  for (int i = 0; i < ns; ++i)
    if (results[i].status > worst) worst = (fe_status)results[i].status;
  return worst;
}

// ---------------------------------------------------------------------------
// float32 batched solve: the float32 iteration of every sample (one launch
// per pass, or one cooperative persistent launch, fe_batch.hip), then the
// float64 verification and, for the samples whose float32 iterate does not
// verify to tol, float64 iterations from that iterate (per-pass launches over
// those samples only)
// ---------------------------------------------------------------------------
struct DevBuffers {
  std::vector<void*> v;
  template <typename P>
  hipError_t alloc(P** p, size_t bytes) {
    void* q = nullptr;
    const hipError_t e = hipMalloc(&q, bytes);
    if (e == hipSuccess) v.push_back(q);
    *p = static_cast<P*>(q);
    return e;
  }
  ~DevBuffers() {
    for (void* q : v) (void)hipFree(q);
  }
};

// samples of one grid: the returned float32 iterates and what the float64
// verification reads
struct F32Class {
  Dims d;
  std::vector<int> ids;
  int ncoef = 1;
  float* eps = nullptr;  // [sample][6][N]
  uint8_t* phase = nullptr;
  PhaseCoef<double>* coef64 = nullptr;
  double* partials = nullptr;  // [sample][bu][7], bu: divergence workgroups per sample (at most)
  int* act = nullptr;
  int bu = 0;
};

// The float32 iteration of every sample in one cooperative launch: grid
// classes cls (at most kBatchClasses, lengths batch_length_ok), iterates
// returned in cls[c].eps with results (status, iterations, eta, mean stress).
static fe_status run_persistent(int op, bool accel, const fe_plan_options& o, const fe_batch_desc* desc, double tol,
                                std::vector<F32Class>& cls, int grid, DevBuffers& mem, fe_batch_result* results,
                                double* seconds) {
  hipStream_t s = (hipStream_t)o.hip_stream;
  BatchDev hb;
  std::memset(&hb, 0, sizeof hb);
  hb.ncls = (int)cls.size();
  hb.tol = tol;
  hb.max_iter = o.max_iter;
  hb.diverge_window = o.diverge_window;
  std::vector<std::vector<float>> host_tables;  // alive until the stream synchronises
  int first = 0;
  for (size_t c = 0; c < cls.size(); ++c) {
    BatchClassDev& C = hb.cls[c];
    const Dims d = cls[c].d;
    const int n = (int)cls[c].ids.size();
    const long long N = d.N;
    const size_t spec = (size_t)spec_size(d);
    C.d = d;
    C.n = n;
    C.nact = n;
    C.first = first;
    first += n;
    C.ncoef = cls[c].ncoef;
    batch_class_layout(d, &C.bz, &C.by, &C.bx, &C.bu, &C.zchunk);
    C.eps[0] = cls[c].eps;
    HIP_TRY(mem.alloc(&C.eps[1], (size_t)n * 6 * N * sizeof(float)));
    HIP_TRY(mem.alloc(&C.R[0], (size_t)n * 3 * N * sizeof(float)));
    HIP_TRY(mem.alloc(&C.R[1], (size_t)n * 3 * N * sizeof(float)));
    HIP_TRY(mem.alloc(&C.S, (size_t)n * 3 * spec * sizeof(cpx<float>)));
    C.phase = cls[c].phase;
    C.partials = cls[c].partials;
    C.act = cls[c].act;
    PhaseCoef<float>* coef = nullptr;
    HIP_TRY(mem.alloc(&coef, (size_t)n * C.ncoef * sizeof(PhaseCoef<float>)));
    C.coef = coef;
    GreenConst<float>* gcon = nullptr;
    HIP_TRY(mem.alloc(&gcon, (size_t)n * sizeof(GreenConst<float>)));
    C.gcon = gcon;
    const int dims[3] = {d.nx, d.ny, d.nz};
    float* wave[3];
    for (int a = 0; a < 3; ++a) {
      std::vector<double> tw = twiddles(dims[a]), wv = wave_table(dims[a], op);
      host_tables.emplace_back(tw.begin(), tw.end());
      host_tables.emplace_back(wv.begin(), wv.end());
      cpx<float>* twd = nullptr;
      HIP_TRY(mem.alloc(&twd, tw.size() * sizeof(float)));
      HIP_TRY(mem.alloc(&wave[a], wv.size() * sizeof(float)));
      HIP_TRY(hipMemcpyAsync(twd, host_tables[host_tables.size() - 2].data(), tw.size() * sizeof(float),
                             hipMemcpyHostToDevice, s));
      HIP_TRY(hipMemcpyAsync(wave[a], host_tables.back().data(), wv.size() * sizeof(float), hipMemcpyHostToDevice,
                             s));
      C.tw[a] = twd;
    }
    C.wt = WaveTables<float>{wave[0], wave[1], wave[2]};
    std::vector<PhaseCoef<float>> cT((size_t)n * C.ncoef);
    std::vector<GreenConst<float>> gv(n);
    std::vector<int> idx(n);
    for (int j = 0; j < n; ++j) {
      const int i = cls[c].ids[j];
      idx[j] = j;
      const fe_materials& m = desc->materials[i];
      const RefMedium ref = reference_medium(o, accel ? FE_ACCELERATED : FE_DIRECT, m);
      std::vector<PhaseCoef<double>> pc = phase_coefs(m, ref);
      for (int q = 0; q < m.n_phases; ++q) {
        PhaseCoef<float>& t = cT[(size_t)j * C.ncoef + q];
        t.lam = float(pc[q].lam);
        t.mu = float(pc[q].mu);
        t.dlam = float(pc[q].dlam);
        t.dmu = float(pc[q].dmu);
        t.ak = float(pc[q].ak);
        t.am = float(pc[q].am);
        t.pad0 = t.pad1 = 0.f;
      }
      GreenConst<float>& g = gv[j];
      g.lam0 = float(ref.lam0);
      g.mu0 = float(ref.mu0);
      g.cr = float((ref.lam0 + ref.mu0) / (ref.lam0 + 2.0 * ref.mu0));
      g.s1 = float(1.0 / (2.0 * ref.mu0));
      g.s2 = float(ref.lam0 / (2.0 * ref.mu0 * (3.0 * ref.lam0 + 2.0 * ref.mu0)));
      g.inv_n = float(1.0 / (double)N);
      for (int q = 0; q < 6; ++q) g.macro[q] = float(desc->macro_strain[6 * i + q]);
      Launch<float>::fill_macro(C.eps[0] + (size_t)j * 6 * N, N, desc->macro_strain + 6 * i, s);
    }
    HIP_TRY(hipMemcpyAsync(coef, cT.data(), cT.size() * sizeof(PhaseCoef<float>), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(gcon, gv.data(), gv.size() * sizeof(GreenConst<float>), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(C.act, idx.data(), idx.size() * sizeof(int), hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));  // the host vectors above go out of scope
  }
  std::vector<BatchState> st(first);
  for (BatchState& x : st) {
    std::memset(&x, 0, sizeof x);
    x.status = kBatchRunning;
    x.prev = INFINITY;
    x.best = INFINITY;
  }
  BatchState* dst = nullptr;
  HIP_TRY(mem.alloc(&dst, st.size() * sizeof(BatchState)));
  HIP_TRY(hipMemcpyAsync(dst, st.data(), st.size() * sizeof(BatchState), hipMemcpyHostToDevice, s));
  hb.st = dst;
  HIP_TRY(mem.alloc(&hb.ctrl, 2 * sizeof(int)));
  HIP_TRY(hipMemsetAsync(hb.ctrl, 0, 2 * sizeof(int), s));
  HIP_TRY(mem.alloc(&hb.bar, sizeof(unsigned long long)));
  HIP_TRY(hipMemsetAsync(hb.bar, 0, sizeof(unsigned long long), s));
  BatchDev* dbd = nullptr;
  HIP_TRY(mem.alloc(&dbd, sizeof(BatchDev)));
  HIP_TRY(hipMemcpyAsync(dbd, &hb, sizeof(BatchDev), hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));

  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  HIP_TRY(hipEventRecord(e0, s));
  HIP_TRY(launch_batch_persistent(op, accel, dbd, grid, s));
  HIP_TRY(hipEventRecord(e1, s));
  HIP_TRY(hipEventSynchronize(e1));
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *seconds = ms * 1e-3;
  int hctrl[2] = {0, 0};
  HIP_TRY(hipMemcpy(hctrl, hb.ctrl, sizeof hctrl, hipMemcpyDeviceToHost));
  if (hctrl[1]) return fail(FE_ERR_DEVICE, "persistent batched solve: a grid barrier timed out");
  HIP_TRY(hipMemcpy(st.data(), dst, st.size() * sizeof(BatchState), hipMemcpyDeviceToHost));
  for (size_t c = 0; c < cls.size(); ++c) {  // results; the final iterate into the returned slot
    const BatchClassDev& C = hb.cls[c];
    const long long N = C.d.N;
    for (int j = 0; j < C.n; ++j) {
      const BatchState& x = st[C.first + j];
      fe_batch_result& r = results[cls[c].ids[j]];
      r.status = x.status == kBatchRunning ? FE_NOT_CONVERGED : x.status;
      r.iterations = x.iterations;
      r.eta = x.eta;
      for (int q = 0; q < 6; ++q) r.mean_stress[q] = x.mean[q];
      if (x.parity)
        HIP_TRY(hipMemcpyAsync(C.eps[0] + (size_t)j * 6 * N, C.eps[1] + (size_t)j * 6 * N, 6 * N * sizeof(float),
                               hipMemcpyDeviceToDevice, s));
    }
  }
  return FE_OK;
}

fe_status solve_batched_f32(int op, bool accel, const fe_plan_options& o, const fe_batch_desc* desc, double tol,
                            fe_batch_result* results, double* seconds) {
  const int ns = desc->n_samples;
  hipStream_t s = (hipStream_t)o.hip_stream;
  std::vector<F32Class> cls;
  for (int i = 0; i < ns; ++i) {
    const fe_grid& g = desc->grids[i];
    size_t c = 0;
    for (; c < cls.size(); ++c)
      if (cls[c].d.nx == g.nx && cls[c].d.ny == g.ny && cls[c].d.nz == g.nz) break;
    if (c == cls.size()) {
      F32Class fc;
      fc.d = make_dims(g.nx, g.ny, g.nz);
      cls.push_back(fc);
    }
    cls[c].ids.push_back(i);
    cls[c].ncoef = std::max(cls[c].ncoef, desc->materials[i].n_phases);
  }
  DevBuffers mem;
  int* flag = nullptr;
  HIP_TRY(mem.alloc(&flag, sizeof(int)));
  HIP_TRY(hipMemsetAsync(flag, 0, sizeof(int), s));
  bool persistent = o.batch_launch == FE_BATCH_PERSISTENT && cls.size() <= (size_t)kBatchClasses;
  for (F32Class& c : cls) {
    const int n = (int)c.ids.size();
    const long long N = c.d.N;
    persistent = persistent && batch_length_ok(c.d.nx) && batch_length_ok(c.d.ny) && batch_length_ok(c.d.nz);
    c.bu = div_partial_count(c.d);
    HIP_TRY(mem.alloc(&c.eps, (size_t)n * 6 * N * sizeof(float)));
    HIP_TRY(mem.alloc(&c.phase, (size_t)n * N));
    HIP_TRY(mem.alloc(&c.coef64, (size_t)n * c.ncoef * sizeof(PhaseCoef<double>)));
    HIP_TRY(mem.alloc(&c.partials, (size_t)n * c.bu * 7 * sizeof(double)));
    HIP_TRY(mem.alloc(&c.act, (size_t)n * sizeof(int)));
    std::vector<PhaseCoef<double>> c64((size_t)n * c.ncoef);
    for (int j = 0; j < n; ++j) {
      const int i = c.ids[j];
      const fe_materials& m = desc->materials[i];
      const RefMedium ref = reference_medium(o, accel ? FE_ACCELERATED : FE_DIRECT, m);
      std::vector<PhaseCoef<double>> pc = phase_coefs(m, ref);
      for (int q = 0; q < m.n_phases; ++q) c64[(size_t)j * c.ncoef + q] = pc[q];
      HIP_TRY(hipMemcpyAsync(c.phase + (size_t)j * N, desc->phase[i], N, hipMemcpyDeviceToDevice, s));
      Launch<float>::check_phase(c.phase + (size_t)j * N, N, m.n_phases, flag, s);
    }
    HIP_TRY(hipMemcpyAsync(c.coef64, c64.data(), c64.size() * sizeof(PhaseCoef<double>), hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  int hflag = 0;
  HIP_TRY(hipMemcpy(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost));
  if (hflag) return fail(FE_ERR_INVALID_ARG, "a phase map holds a label >= its n_phases");
  const int grid = persistent ? batch_persistent_grid(op, accel) : 0;
  if (persistent && grid <= 0) return fail(FE_ERR_UNSUPPORTED, "cooperative launches are not available");

  // the float32 iteration; iterates into cls[c].eps
  double sec32 = 0.0;
  if (persistent) {
    fe_status ps = run_persistent(op, accel, o, desc, tol, cls, grid, mem, results, &sec32);
    if (ps != FE_OK) return ps;
  } else {
    std::vector<void*> slot(ns);
    for (const F32Class& c : cls)
      for (size_t j = 0; j < c.ids.size(); ++j) slot[c.ids[j]] = c.eps + j * 6 * c.d.N;
    fe_batch_desc sd = *desc;
    sd.strain = slot.data();
    const fe_status st32 = solve_batched_impl<float>(op, accel, o, &sd, tol, results, &sec32);
    if (st32 < 0) return st32;
  }
  if (seconds) *seconds = sec32;

  // float64 verification of the float32 strains
  double* red = nullptr;
  HIP_TRY(mem.alloc(&red, (size_t)std::max(ns, 1) * 8 * sizeof(double)));
  auto verify = [&](F32Class& c, std::vector<double>& out) -> fe_status {
    const int n = (int)c.ids.size();
    const Batch bt{c.act, c.ncoef};
    std::vector<int> all(n);
    for (int j = 0; j < n; ++j) all[j] = j;
    HIP_TRY(hipMemcpyAsync(c.act, all.data(), all.size() * sizeof(int), hipMemcpyHostToDevice, s));
    const int nb = launch_div64<float>(c.eps, c.phase, c.coef64, nullptr, nullptr, c.partials, c.d, op, s, bt, n);
    launch_reduce(c.partials, nb, 7, red, s, c.act, n);
    std::vector<double> h((size_t)n * 8);
    HIP_TRY(hipMemcpyAsync(h.data(), red, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    out.resize(n);
    for (int j = 0; j < n; ++j) {
      double mean[6];
      for (int q = 0; q < 6; ++q) mean[q] = h[8 * j + 1 + q] / (double)c.d.N;
      out[j] = std::sqrt(h[8 * j] / (double)c.d.N) / frob(mean);
    }
    return FE_OK;
  };
  // samples whose float32 strain does not verify: float64 iterations from it
  std::vector<std::pair<int, int>> redo;  // (class, index in class)
  for (size_t c = 0; c < cls.size(); ++c) {
    std::vector<double> ev;
    fe_status vs = verify(cls[c], ev);
    if (vs != FE_OK) return vs;
    for (size_t j = 0; j < cls[c].ids.size(); ++j) {
      fe_batch_result& r = results[cls[c].ids[j]];
      r.eta_verify_fp64 = ev[j];
      if (o.refine && r.status != FE_DIVERGED && !(ev[j] <= tol) && r.iterations < o.max_iter)
        redo.emplace_back((int)c, (int)j);
    }
  }
  // A continuation that reached its target in float64 can still miss tol once
  // its strain is rounded to float32; such samples continue again from the
  // rounded strain with the target halved (at most four times, and only while
  // the verified eta keeps falling).
  double target = tol;
  for (int lowered = 0; !redo.empty(); ++lowered) {
    const int nr = (int)redo.size();
    std::vector<fe_grid> grids(nr);
    std::vector<const uint8_t*> phases(nr);
    std::vector<fe_materials> mats(nr);
    std::vector<double> macro((size_t)6 * nr);
    std::vector<void*> out64(nr);
    std::vector<const float*> init(nr);
    std::vector<fe_batch_result> sub(nr);
    for (int k = 0; k < nr; ++k) {
      const F32Class& c = cls[redo[k].first];
      const int j = redo[k].second, i = c.ids[j];
      grids[k] = desc->grids[i];
      phases[k] = desc->phase[i];
      mats[k] = desc->materials[i];
      for (int q = 0; q < 6; ++q) macro[6 * k + q] = desc->macro_strain[6 * i + q];
      double* o64 = nullptr;
      HIP_TRY(mem.alloc(&o64, (size_t)6 * c.d.N * sizeof(double)));
      out64[k] = o64;
      init[k] = c.eps + (size_t)j * 6 * c.d.N;
    }
    fe_batch_desc sd;
    sd.n_samples = nr;
    sd.grids = grids.data();
    sd.phase = phases.data();
    sd.materials = mats.data();
    sd.macro_strain = macro.data();
    sd.strain = out64.data();
    fe_plan_options o64 = o;
    o64.precision = FE_FP64;
    double sec64 = 0.0;
    const fe_status st64 = solve_batched_impl<double>(op, accel, o64, &sd, target, sub.data(), &sec64, init.data());
    if (st64 < 0) return st64;
    if (seconds) *seconds += sec64;
    for (int k = 0; k < nr; ++k) {
      const F32Class& c = cls[redo[k].first];
      const int j = redo[k].second;
      Launch<float>::convert_to(c.eps + (size_t)j * 6 * c.d.N, out64[k], 1, 6 * c.d.N, s);
      fe_batch_result& r = results[c.ids[j]];
      r.iterations += sub[k].iterations;
      r.eta = sub[k].eta;
      for (int q = 0; q < 6; ++q) r.mean_stress[q] = sub[k].mean_stress[q];
      r.status = sub[k].status;
    }
    std::vector<double> last(nr);
    for (int k = 0; k < nr; ++k) last[k] = results[cls[redo[k].first].ids[redo[k].second]].eta_verify_fp64;
    for (F32Class& c : cls) {  // the returned float32 strains, verified again
      std::vector<double> ev;
      fe_status vs = verify(c, ev);
      if (vs != FE_OK) return vs;
      for (size_t j = 0; j < c.ids.size(); ++j) results[c.ids[j]].eta_verify_fp64 = ev[j];
    }
    std::vector<std::pair<int, int>> again;
    for (int k = 0; k < nr; ++k) {
      const fe_batch_result& r = results[cls[redo[k].first].ids[redo[k].second]];
      if (r.status == FE_OK && !(r.eta_verify_fp64 <= tol) && r.eta_verify_fp64 < 0.9 * last[k] &&
          r.iterations < o.max_iter && lowered < 4)
        again.push_back(redo[k]);
    }
    redo.swap(again);
    target *= 0.5;
  }
  // with refinement FE_OK means the returned float32 strain verifies to tol
  // (a sample that cannot continue, or ends at the float32 storage floor of
  // its rounded strain, is FE_NOT_CONVERGED)
  if (o.refine)
    for (int i = 0; i < ns; ++i)
      if (results[i].status == FE_OK && !(results[i].eta_verify_fp64 <= tol)) results[i].status = FE_NOT_CONVERGED;
  for (const F32Class& c : cls)
    for (size_t j = 0; j < c.ids.size(); ++j) {
      const int i = c.ids[j];
      if (desc->strain && desc->strain[i])
        HIP_TRY(hipMemcpyAsync(desc->strain[i], c.eps + j * 6 * c.d.N, 6 * c.d.N * sizeof(float),
                               hipMemcpyDeviceToDevice, s));
    }
  HIP_TRY(hipStreamSynchronize(s));
  fe_status worst = FE_OK;
  for (int i = 0; i < ns; ++i)
    if (results[i].status > worst) worst = (fe_status)results[i].status;
  return worst;
}

}  // namespace

extern "C" fe_status fe_solve_batched(fe_discretization disc, fe_scheme scheme, const fe_plan_options* opt,
                                      const fe_batch_desc* desc, double tol, fe_batch_result* results,
                                      double* seconds) {
  if (!desc || !results) return fail(FE_ERR_INVALID_ARG, "desc or results is NULL");
  if (disc != FE_GREEN_WP && disc != FE_GREEN_ROT)
    return fail(disc == FE_GREEN_MS || disc == FE_GREEN_CENTERED || disc == FE_GREEN_MS_SYMMETRIZED
                    ? FE_ERR_UNSUPPORTED
                    : FE_ERR_INVALID_ARG,
                "batched solves support the WP and ROT operators");
  if (scheme == FE_CONJUGATE_GRADIENT)
    return fail(FE_ERR_UNSUPPORTED, "batched solves run the direct and accelerated schemes");
  if (scheme != FE_DIRECT && scheme != FE_ACCELERATED) return fail(FE_ERR_INVALID_ARG, "unknown scheme");
  fe_plan_options o;
  fe_plan_options_default(&o);
  if (opt) {
    if (opt->struct_size != sizeof(fe_plan_options)) return fail(FE_ERR_INVALID_ARG, "bad fe_plan_options.struct_size");
    o = *opt;
  }
  if (o.precision != FE_FP32 && o.precision != FE_FP64) return fail(FE_ERR_INVALID_ARG, "unknown precision");
  if (o.max_iter < 0) return fail(FE_ERR_INVALID_ARG, "max_iter must be >= 0");
  if (o.ref_rule == FE_REF_EXPLICIT &&
      !(std::isfinite(o.E0) && o.E0 > 0.0 && std::isfinite(o.nu0) && o.nu0 > -1.0 && o.nu0 < 0.5))
    return fail(FE_ERR_INVALID_ARG, "explicit reference needs E0 > 0 and -1 < nu0 < 0.5");
  if (!(tol > 0.0) || !std::isfinite(tol)) return fail(FE_ERR_INVALID_ARG, "tol must be finite and > 0");
  if (desc->n_samples < 1 || desc->n_samples > 65535) return fail(FE_ERR_INVALID_ARG, "n_samples must be in [1, 65535]");
  if (!desc->grids || !desc->phase || !desc->materials || !desc->macro_strain)
    return fail(FE_ERR_INVALID_ARG, "desc arrays are NULL");
  for (int i = 0; i < desc->n_samples; ++i) {
    const fe_grid& g = desc->grids[i];
    const int n[3] = {g.nx, g.ny, g.nz};
    for (int a = 0; a < 3; ++a)
      if (!(a == 2 ? supported_z_length(n[a]) : supported_length(n[a])))
        return fail(FE_ERR_UNSUPPORTED, "sample %d: grid dimension %d = %d", i, a, n[a]);
    if (!desc->phase[i]) return fail(FE_ERR_INVALID_ARG, "sample %d: phase is NULL", i);
    fe_status st = validate_materials(desc->materials[i]);
    if (st != FE_OK) return st;
    for (int q = 0; q < 6; ++q)
      if (!std::isfinite(desc->macro_strain[6 * i + q])) return fail(FE_ERR_INVALID_ARG, "sample %d: macro strain", i);
  }
  const int op = disc == FE_GREEN_WP ? OP_WP : OP_ROT;
  if (o.batch_launch != FE_BATCH_PER_PASS && o.batch_launch != FE_BATCH_PERSISTENT)
    return fail(FE_ERR_INVALID_ARG, "unknown batch_launch");
  if (o.precision == FE_FP64) {
    if (o.batch_launch == FE_BATCH_PERSISTENT)
      return fail(FE_ERR_UNSUPPORTED, "the persistent batched launch runs float32 fields");
    return solve_batched_impl<double>(op, scheme == FE_ACCELERATED, o, desc, tol, results, seconds);
  }
  return solve_batched_f32(op, scheme == FE_ACCELERATED, o, desc, tol, results, seconds);
}
