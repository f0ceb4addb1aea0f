// Host-side launchers of the gfx950 kernels (one instantiation per real type).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fe_device.h"

namespace fe {

// OP_MSS: the continuous operator with eq. (15)'s symmetrised Nyquist rule
// in place of eq. (14)'s (C0)^-1
enum Op { OP_MS = 0, OP_WP = 1, OP_ROT = 2, OP_C = 3, OP_MSS = 4 };

struct Dims {
  int nx, ny, nz, H;  // H = nz/2 + 1 (half spectrum along z)
  long long N;        // nx*ny*nz
  int zs;             // the transform work buffers group z in blocks of 2^zs planes
  int Hp;             // half-spectrum planes stored: H rounded up to 2^zs
};

// Grid dimensions with the z blocking of the transform work buffers: blocks
// of 8 planes where nz allows (else the largest power of two dividing nz).
inline Dims make_dims(int nx, int ny, int nz) {
  Dims d;
  d.nx = nx;
  d.ny = ny;
  d.nz = nz;
  d.H = nz / 2 + 1;
  d.N = (long long)nx * ny * nz;
  d.zs = 3;
  while (d.zs > 0 && nz % (1 << d.zs) != 0) --d.zs;
  d.Hp = ((d.H + (1 << d.zs) - 1) >> d.zs) << d.zs;
  return d;
}

// Layout of the transform work buffers (divergence / displacement planes,
// six-component polarization planes, half spectra): row (z, y) of a component
// sits at ((z >> zs) ny + y) 2^zs + (z mod 2^zs), x fastest.  A column along z
// then crosses nz / 2^zs page-sized strides instead of nz (address
// translation: one 2 MiB page per plane at 1024^2 planes).  The strain, phase
// and stress fields keep the plain [z][y][x] layout.
__host__ __device__ __forceinline__ long long zrow(const Dims& d, int z, int y) {
  return (((long long)(z >> d.zs) * d.ny + y) << d.zs) + (z & ((1 << d.zs) - 1));
}
// element of the blocked layout holding plain voxel (z, y, x)
__host__ __device__ __forceinline__ long long zidx(const Dims& d, int z, int y, int x) {
  return zrow(d, z, y) * d.nx + x;
}
// plain voxel index v = (z ny + y) nx + x -> blocked element
__host__ __device__ __forceinline__ long long zblk(const Dims& d, long long v) {
  if (d.zs == 0) return v;
  const long long zy = v / d.nx;
  return zidx(d, (int)(zy / d.ny), (int)(zy % d.ny), (int)(v - zy * d.nx));
}
// half-spectrum values per component (padded planes included)
__host__ __device__ __forceinline__ long long spec_size(const Dims& d) { return (long long)d.Hp * d.ny * d.nx; }

// Per-phase constants derived on the host in float64 from (E, nu) and C0.
template <typename T>
struct PhaseCoef {
  T lam, mu;    // C = lam I(x)I + 2 mu Id
  T dlam, dmu;  // C - C0
  T ak, am;     // 2 kappa0/(kappa+kappa0), 2 mu0/(mu+mu0): (C+C0)^-1 C0 times 2
  T pad0, pad1;
};

// Reference-medium constants of the Green operator.
template <typename T>
struct GreenConst {
  T lam0, mu0;
  T cr;       // (lam0 + mu0)/(lam0 + 2 mu0)
  T s1, s2;   // (C0)^-1 : tau = s1 tau - s2 tr(tau) I
  T inv_n;    // 1/N, folded into the Green step so inverse transforms are unnormalised
  T macro[6]; // eps_bar (tensor Voigt order)
};

// Batched launches: blockIdx.y selects a slot of the active-sample list; every
// per-sample buffer of a size class is packed with a fixed stride (strain 6N,
// phase N, real work planes ncomp*N, half spectra ncomp*Hp*ny*nx, partial sums
// gridDim.x*7, phase constants ncoef).
struct Batch {
  const int* active;  // null: a single sample (sample 0)
  int ncoef;          // PhaseCoef entries per sample
};

// Per-axis wave tables, 2 reals per index m in [0, n):
//   ROT: (sin(pi m'/n), cos(pi m'/n));  WP: (cos q - 1, sin q);  MS: (q, 1 if Nyquist else 0)
template <typename T>
struct WaveTables {
  const T* x;
  const T* y;
  const T* z;
};

template <typename T>
struct Launch {
  // eps^0 = eps_bar
  static void fill_macro(T* eps, long long N, const double* macro, hipStream_t s);
  static void convert_to(T* dst, const void* src, int src_is_double, long long n, hipStream_t s);
  static void check_phase(const uint8_t* phase, long long N, int n_phases, int* flag, hipStream_t s);

  // Displacement form (WP and ROT operators).
  // Writes the divergence of tau to D; Dsig_base (nullable) is added to the
  // divergence of sigma before eta's reduction.  Returns the number of partial
  // sums (7 doubles each) written.
  static int div(const T* eps, const uint8_t* phase, const PhaseCoef<T>* coef, T* D, const T* Dsig_base,
                 double* partials, Dims d, int op, hipStream_t s, Batch bt = Batch{nullptr, 0}, int nsamp = 1);
  // Strain update then div in one walk: eps_out = update(U, eps_in) and D =
  // div tau(eps_out) with eta's partial sums (eps_out nullable: not written, and the first of the seven sums
  // is then U.D over the owned corners instead of |div sigma|^2); eps_in and eps_out must not
  // overlap.  rfield (nullable, 6 planes) replaces the constant applied
  // strain; gs (nullable) holds per-sample constants that replace g.  Returns
  // the number of partial sums (same tiling as div).
  static int update_div(const T* U, const T* eps_in, T* eps_out, const uint8_t* phase, const PhaseCoef<T>* coef,
                        GreenConst<T> g, const T* rfield, T* D, const T* Dsig_base, double* partials, Dims d,
                        int op, int accelerated, hipStream_t s, Batch bt = Batch{nullptr, 0},
                        const GreenConst<T>* gs = nullptr, int nsamp = 1);
  static void axpy(T* y, const T* x, long long n, hipStream_t s);  // y += x
  // Conjugate gradients (displacement form; scalars in cgs, see k_cg_step).
  // dot and cg_step return the number of partial sums (one double each).
  static int dot(const T* a, const T* b, long long n, double* partials, hipStream_t s);
  static int cg_step(T* v, const T* p, T* r, const T* Q, long long n, double* cgs, double* partials, hipStream_t s);
  static void cg_dir(T* p, const T* z, long long n, const double* cgs, int first, hipStream_t s);
  // Six-component conjugate gradients (inner product sum a:C0:b, see
  // k_cg6_step): Q = (negate ? -1 : 1) Rb taken out of the z-blocked layout,
  // with the partial sums of <x, Q> (x nullable: <Q, Q>); the step
  // eps += alpha p, r -= alpha Q with the partial sums of <r, r>.  Both
  // return the number of partial sums (one double each).
  static int cg6_take(const T* Rb, T* Q, const T* x, int negate, Dims d, double lam0, double mu0, double* partials,
                      hipStream_t s);
  static int cg6_step(T* eps, const T* p, T* r, const T* Q, long long N, double lam0, double mu0, double* cgs,
                      double* partials, hipStream_t s);
  static void xgreen3(cpx<T>* S, Dims d, const cpx<T>* twx, WaveTables<T> wt, GreenConst<T> g, int op,
                      hipStream_t s, Batch bt = Batch{nullptr, 0}, const GreenConst<T>* gs = nullptr, int nsamp = 1);

  // Six-component form (every operator).
  static void tau6(const T* eps, const uint8_t* phase, const PhaseCoef<T>* coef, T* out, int write_sigma,
                   double* partials, int nblocks, Dims d, hipStream_t s);
  static void xgreen6(cpx<T>* S, Dims d, const cpx<T>* twx, WaveTables<T> wt, GreenConst<T> g, int op,
                      hipStream_t s);
  // Returns the number of partial sums written.
  static int xeta6(const cpx<T>* S, Dims d, const cpx<T>* twx, WaveTables<T> wt, double* partials, int op,
                   hipStream_t s);
  // e (the inverse transform output) plus rfield (nullable, plain [6][N]:
  // the anchor's strain residual replacing the applied strain) updates eps
  static void update6(const T* e, T* eps, const uint8_t* phase, const PhaseCoef<T>* coef, Dims d,
                      int accelerated, hipStream_t s, const T* rfield = nullptr);

  // Strided FFT passes.
  static void zr2c(const T* R, cpx<T>* S, int ncomp, Dims d, const cpx<T>* twz, hipStream_t s,
                   Batch bt = Batch{nullptr, 0}, int nsamp = 1);
  static void zc2r(const cpx<T>* S, T* R, int ncomp, Dims d, const cpx<T>* twz, hipStream_t s,
                   Batch bt = Batch{nullptr, 0}, int nsamp = 1);
  static void yfft(cpx<T>* S, int ncomp, Dims d, const cpx<T>* twy, int inverse, hipStream_t s,
                   Batch bt = Batch{nullptr, 0}, int nsamp = 1);

  static void stress(const T* eps, const uint8_t* phase, const PhaseCoef<T>* coef, T* sigma, long long N,
                     hipStream_t s);
};

enum { XETA_PLAIN = 0, XETA_BASE = 1, XETA_STORE = 2 };
// Spectral eta of the six-component form (mode XETA_PLAIN, XETA_BASE,
// XETA_STORE of fe_passes.h; base: the anchor's divergence spectrum, 6 half
// spectra of TS, read by XETA_BASE and written by XETA_STORE; these two
// modes take OP_MS or OP_C).  Returns the number of partial sums written.
template <typename T, typename TS>
int launch_xeta6(const cpx<T>* S, Dims d, const cpx<T>* twx, WaveTables<T> wt, double* partials, int op, int mode,
                 cpx<TS>* base, hipStream_t s);

// r = e_hi - eps (r and eps plain [6][N] of TE, e_hi the float64 inverse
// transform output in the z-blocked layout): the six-component anchor's
// strain residual.
template <typename TE>
void launch_residual6(const double* e_hi, const TE* eps, TE* r, Dims d, hipStream_t s);

// Conjugate gradients: |r|^2 and the sums of sigma taken from the last fused
// gradient/divergence launch's reduced sums (cgs[16..22]).
void launch_cg_restart(double* cgs, hipStream_t s);

// float64 verification of eta from a strain of storage type TS (ROT, WP).
// Returns the number of partial sums (7 doubles each) written.
template <typename TS>
int launch_verify_div(const TS* eps, const uint8_t* phase, const PhaseCoef<double>* coef, double* partials, Dims d,
                      int op, hipStream_t s);

// float64 divergences of an anchor strain: Dtau (float64, nullable) and Dsig
// (storage type, nullable); partial sums as in Launch::div.
template <typename TS>
int launch_div64(const TS* eps, const uint8_t* phase, const PhaseCoef<double>* coef, double* Dtau, TS* Dsig,
                 double* partials, Dims d, int op, hipStream_t s, Batch bt = Batch{nullptr, 0}, int nsamp = 1);

// r = eps_bar + sym grad_h U - eps in float64 arithmetic (U float64).
template <typename TE>
void launch_residual(const double* U, const TE* eps, GreenConst<double> g, TE* r, Dims d, int op, hipStream_t s);

// Upper bound on the partial sums (per sample) a divergence launch over grid d
// writes, float or double tiles; the launchers return the exact count.
int div_partial_count(Dims d);

// Fixed-order sums of per-block partials: out[8*sample + i] for i < nv; with an
// active list, one reduction per active sample (partials strided by nblocks*nv).
void launch_reduce(const double* partials, int nblocks, int nv, double* out, hipStream_t s,
                   const int* active = nullptr, int nsamp = 1);

constexpr int kThreads = 256;
constexpr int kMaxReduceBlocks = 16384;

}  // namespace fe
