// gfx950 kernels of the Lippmann-Schwinger FFT iteration (Willot, arXiv
// 1412.8398).  Equation numbers refer to the paper.
//
// Layouts: real fields are SoA planes [comp][z][y][x] of N = nx*ny*nz values;
// spectra are half spectra along z: [comp][mz][y][x] complex, mz in [0, nz/2].
// Tensor components use Voigt order (11, 22, 33, 23, 13, 12).
#include <type_traits>

#include "fe_stencil.h"

namespace fe {

// --------------------------------------------------------------------------
// initialisation, checks, conversions
// --------------------------------------------------------------------------

template <typename T>
__global__ void k_fill_macro(T* __restrict__ eps, long long N, T m0, T m1, T m2, T m3, T m4, T m5) {
  const T m[6] = {m0, m1, m2, m3, m4, m5};
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N; i += (long long)gridDim.x * blockDim.x) {
#pragma unroll
    for (int c = 0; c < 6; ++c) eps[c * N + i] = m[c];
  }
}

template <typename T, typename S>
__global__ void k_convert(T* __restrict__ dst, const S* __restrict__ src, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    dst[i] = T(src[i]);
}

__global__ void k_check_phase(const uint8_t* __restrict__ phase, long long N, int n_phases, int* flag) {
  int bad = 0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N; i += (long long)gridDim.x * blockDim.x)
    bad |= (phase[i] >= n_phases);
  if (bad) atomicOr(flag, 1);
}

static int grid_for(long long n, int cap = 8192) {
  long long b = (n + kThreads - 1) / kThreads;
  if (b > cap) b = cap;
  if (b < 1) b = 1;
  return (int)b;
}

template <int DX, int DY, typename TS, typename TC, typename TD, int OP>
__global__ __launch_bounds__(DX * DY) void k_div(const TS* __restrict__ eps, const uint8_t* __restrict__ phase,
                                                 const PhaseCoef<TC>* __restrict__ coef, TD* __restrict__ Dtau,
                                                 TS* __restrict__ Dsig, const TS* __restrict__ Dsig_base,
                                                 double* __restrict__ partials, Dims d, int zchunk, Batch bt) {
  {
    const long long smp = bt.active ? bt.active[blockIdx.y] : 0;
    eps += smp * 6 * d.N;
    phase += smp * d.N;
    coef += smp * bt.ncoef;
    if (Dtau) Dtau += smp * 3 * d.N;
    if (Dsig) Dsig += smp * 3 * d.N;
    if (Dsig_base) Dsig_base += smp * 3 * d.N;
    partials += smp * gridDim.x * 7;
  }
  __shared__ DivLds<TC, DX, DY> L;
  div_body<DX, DY, TS, TC, TD, OP>(L, eps, phase, coef, Dtau, Dsig, Dsig_base, partials + blockIdx.x * 7, d, zchunk,
                                   xcd_block(blockIdx.x, gridDim.x));
}

template <int DX, int DY, typename T, int OP, bool AS, bool RF, bool WE>
__global__ __launch_bounds__(DX * DY) void k_update_div(const T* __restrict__ U, const T* __restrict__ eps_in,
                                                        T* __restrict__ eps_out, const uint8_t* __restrict__ phase,
                                                        const PhaseCoef<T>* __restrict__ coef, int ncoef,
                                                        GreenConst<T> g, const T* __restrict__ rfield,
                                                        T* __restrict__ Dtau, const T* __restrict__ Dsig_base,
                                                        double* __restrict__ partials, Dims d, int zchunk, Batch bt,
                                                        const GreenConst<T>* __restrict__ gs) {
  const long long N = d.N;
  {
    const long long smp = bt.active ? bt.active[blockIdx.y] : 0;
    U += smp * 3 * N;
    eps_in += smp * 6 * N;
    if (WE) eps_out += smp * 6 * N;
    phase += smp * N;
    coef += smp * bt.ncoef;
    if (RF) rfield += smp * 6 * N;
    Dtau += smp * 3 * N;
    if (Dsig_base) Dsig_base += smp * 3 * N;
    partials += smp * gridDim.x * 7;
    if (gs) g = gs[smp];
  }
  __shared__ UpdLds<T, DX, DY> L;
  update_div_body<DX, DY, T, OP, AS, RF, WE>(L, U, eps_in, eps_out, phase, coef, ncoef, g, rfield, Dtau, Dsig_base,
                                             partials + blockIdx.x * 7, d, zchunk, xcd_block(blockIdx.x, gridDim.x));
}

int div_partial_count(Dims d) {
  // the smallest tiles give the most workgroups (grids up to 128 wide and the
  // float64 verification use 32 x 8; wider grids 128 x 8, or 64 x 8 in float64)
  return div_grid<Tile<float>::DX, Tile<float>::DY>(d).blocks > div_grid<32, 8>(d).blocks
             ? div_grid<Tile<float>::DX, Tile<float>::DY>(d).blocks
             : div_grid<32, 8>(d).blocks;
}

// --------------------------------------------------------------------------
// strain update from the displacement U (WP, ROT)
// ROT: grad at voxel v from its corners v + a: d_i U_j = 1/4 sum_a s_i(a) U_j(v+a),
// s_i(a) = +1 if a_i = 1 else -1 (eq. (37)), symbol k^R.
// WP: forward differences d_i U_j = U_j(v + e_i) - U_j(v) (eq. (23)), symbol k^W.
// e = eps_bar + sym grad U;  DS (eq. (9)): eps <- e;
// AS (eq. (16)): eps <- eps + 2 kappa0/(kappa+kappa0) sph(e - eps) + 2 mu0/(mu+mu0) dev(e - eps).
// --------------------------------------------------------------------------

// Strain residual of an anchor strain in float64 arithmetic:
// r = eps_bar + sym grad_h U - eps (U from the float64 transforms of the
// divergence of (C - C0):eps), stored in the anchor's precision.
template <typename TE, int OP>
__global__ __launch_bounds__(256) void k_residual(const double* __restrict__ U, const TE* __restrict__ eps,
                                                  GreenConst<double> g, TE* __restrict__ r, Dims d) {
  const long long N = d.N;
  const int nx = d.nx, ny = d.ny, nz = d.nz;
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < N; v += (long long)gridDim.x * blockDim.x) {
    const int x = (int)(v % nx);
    const int y = (int)((v / nx) % ny);
    const int z = (int)(v / ((long long)nx * ny));
    double gr[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) gr[i][j] = 0.0;
    if (OP == OP_ROT) {
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        const int ax = a & 1, ay = (a >> 1) & 1, az = (a >> 2) & 1;
        const long long c = zidx(d, wrap(z + az, nz), wrap(y + ay, ny), wrap(x + ax, nx));  // z-blocked U
        const double u[3] = {U[c], U[N + c], U[2 * N + c]};
        const double sg[3] = {ax ? 1.0 : -1.0, ay ? 1.0 : -1.0, az ? 1.0 : -1.0};
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int j = 0; j < 3; ++j) gr[i][j] += sg[i] * u[j];
      }
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) gr[i][j] *= 0.25;
    } else {
      const long long c0 = zidx(d, z, y, x);  // z-blocked U
      const double u0[3] = {U[c0], U[N + c0], U[2 * N + c0]};
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const int xp = i == 0 ? wrap(x + 1, nx) : x;
        const int yp = i == 1 ? wrap(y + 1, ny) : y;
        const int zp = i == 2 ? wrap(z + 1, nz) : z;
        const long long c = zidx(d, zp, yp, xp);
#pragma unroll
        for (int j = 0; j < 3; ++j) gr[i][j] = U[j * N + c] - u0[j];
      }
    }
    const double e[6] = {g.macro[0] + gr[0][0], g.macro[1] + gr[1][1], g.macro[2] + gr[2][2],
                         g.macro[3] + 0.5 * (gr[1][2] + gr[2][1]), g.macro[4] + 0.5 * (gr[0][2] + gr[2][0]),
                         g.macro[5] + 0.5 * (gr[0][1] + gr[1][0])};
#pragma unroll
    for (int k = 0; k < 6; ++k) r[k * N + v] = TE(e[k] - double(eps[k * N + v]));
  }
}

template <typename T>
__global__ void k_axpy(T* __restrict__ y, const T* __restrict__ x, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    y[i] += x[i];
}

// --------------------------------------------------------------------------
// Conjugate gradients on the corner displacement (displacement form).  The
// scalars live on the device (cgs, doubles), so no iteration waits for the
// host: 0 rho = r.z, 1 the previous rho, 3 |r|^2 summed over corners,
// 10..15 the voxel sums of sigma of the current iterate, 16..22 the seven
// reduced sums of the last fused gradient/divergence launch: |div sigma|^2
// (with the strain written) or p.Q with Q = div sigma(grad p) = -K p (without),
// then the six sums of sigma.
// --------------------------------------------------------------------------
constexpr int kCgBlocks = 1024;

template <typename T>
__global__ __launch_bounds__(256) void k_dot3(const T* __restrict__ a, const T* __restrict__ b, long long n,
                                              double* __restrict__ partials) {
  __shared__ double red[16];
  double acc[1] = {0.0};
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
    acc[0] += double(a[i]) * double(b[i]);
  block_sum<1>(acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = acc[0];
}

// alpha = rho / (p.K p) = rho / (-p.Q); v += alpha p; r -= alpha K p = r + alpha Q;
// partial sums of |r|^2.  Block 0 also moves rho to the previous-rho slot and
// adds alpha times the sums of sigma(grad p) to those of the iterate (no
// other block touches those slots).
template <typename T>
__global__ __launch_bounds__(256) void k_cg_step(T* __restrict__ v, const T* __restrict__ p, T* __restrict__ r,
                                                 const T* __restrict__ Q, long long n, double* __restrict__ cgs,
                                                 double* __restrict__ partials) {
  __shared__ double red[16];
  const double alpha = cgs[0] / -cgs[16];
  const T a = T(alpha);
  double acc[1] = {0.0};
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
    v[i] += a * p[i];
    const T ri = r[i] + a * Q[i];
    r[i] = ri;
    acc[0] += double(ri) * double(ri);
  }
  block_sum<1>(acc, red);
  if (threadIdx.x == 0) {
    partials[blockIdx.x] = acc[0];
    if (blockIdx.x == 0) {
      cgs[1] = cgs[0];
      for (int k = 0; k < 6; ++k) cgs[10 + k] += alpha * cgs[17 + k];
    }
  }
}

// Conjugate gradients in the six-component form (strain iterate, inner
// product <a, b> = sum_x a : C0 : b with a : C0 : b = lam0 tr a tr b
// + 2 mu0 (sum_i a_ii b_ii + 2 sum_{i<j} a_ij b_ij), tensor Voigt planes).
template <typename T>
__device__ __forceinline__ double c0_dot(const double* a, const double* b, double lam0, double mu0) {
  return lam0 * (a[0] + a[1] + a[2]) * (b[0] + b[1] + b[2]) +
         2.0 * mu0 * (a[0] * b[0] + a[1] * b[1] + a[2] * b[2] + 2.0 * (a[3] * b[3] + a[4] * b[4] + a[5] * b[5]));
}

// Q = sgn * Rb (Rb: the inverse transform output, z-blocked; Q plain) and the
// partial sums of <x, Q> (x nullable: then <Q, Q>).
template <typename T>
__global__ __launch_bounds__(256) void k_cg6_take(const T* __restrict__ Rb, T* __restrict__ Q, const T* __restrict__ x,
                                                  T sgn, Dims d, double lam0, double mu0,
                                                  double* __restrict__ partials) {
  __shared__ double red[16];
  const long long N = d.N;
  double acc[1] = {0.0};
  for (long long v = blockIdx.x * 256LL + threadIdx.x; v < N; v += (long long)gridDim.x * 256) {
    const long long vb = zblk(d, v);
    double q[6], a[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const T qk = sgn * Rb[k * N + vb];
      Q[k * N + v] = qk;
      q[k] = double(qk);
      a[k] = x ? double(x[k * N + v]) : q[k];
    }
    acc[0] += c0_dot<T>(a, q, lam0, mu0);
  }
  block_sum<1>(acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = acc[0];
}

// alpha = <r, r> / <p, Q> (cgs[0], cgs[16]); eps += alpha p; r -= alpha Q;
// partial sums of <r, r>.  Block 0 moves <r, r> to the previous slot cgs[1].
template <typename T>
__global__ __launch_bounds__(256) void k_cg6_step(T* __restrict__ eps, const T* __restrict__ p, T* __restrict__ r,
                                                  const T* __restrict__ Q, long long N, double lam0, double mu0,
                                                  double* __restrict__ cgs, double* __restrict__ partials) {
  __shared__ double red[16];
  const T a = T(cgs[0] / cgs[16]);
  double acc[1] = {0.0};
  for (long long v = blockIdx.x * 256LL + threadIdx.x; v < N; v += (long long)gridDim.x * 256) {
    double rr[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      eps[k * N + v] += a * p[k * N + v];
      const T rk = r[k * N + v] - a * Q[k * N + v];
      r[k * N + v] = rk;
      rr[k] = double(rk);
    }
    acc[0] += c0_dot<T>(rr, rr, lam0, mu0);
  }
  block_sum<1>(acc, red);
  if (threadIdx.x == 0) {
    partials[blockIdx.x] = acc[0];
    if (blockIdx.x == 0) cgs[1] = cgs[0];
  }
}

// p = z + beta p, beta = rho / previous rho (p = z when first)
template <typename T>
__global__ __launch_bounds__(256) void k_cg_dir(T* __restrict__ p, const T* __restrict__ z, long long n,
                                                const double* __restrict__ cgs, int first) {
  const T beta = first ? T(0) : T(cgs[0] / cgs[1]);
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
    p[i] = first ? z[i] : z[i] + beta * p[i];
}

// restart: |r|^2 and the sums of sigma from the last fused launch's sums
__global__ void k_cg_restart(double* __restrict__ cgs) {
  if (threadIdx.x == 0) {
    cgs[3] = cgs[16];
    for (int k = 0; k < 6; ++k) cgs[10 + k] = cgs[17 + k];
  }
}

// --------------------------------------------------------------------------
// pointwise polarization / stress (6-component form) and update
// --------------------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(256) void k_tau6(const T* __restrict__ eps, const uint8_t* __restrict__ phase,
                                              const PhaseCoef<T>* __restrict__ coef, T* __restrict__ out,
                                              int write_sigma, double* __restrict__ partials, Dims d) {
  const long long N = d.N;
  __shared__ double red[7 * 16];
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < N; v += (long long)gridDim.x * blockDim.x) {
    T e[6];
    load6(eps, N, v, e);
    const PhaseCoef<T> pc = coef[phase[v]];
    T s[6], t[6];
    iso_apply(pc.lam, pc.mu, e, s);
    iso_apply(pc.dlam, pc.dmu, e, t);
    const long long vb = zblk(d, v);  // the transform input: z-blocked
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      out[k * N + vb] = write_sigma ? s[k] : t[k];
      acc[1 + k] += double(s[k]);
    }
  }
  if (partials) {
    block_sum<7>(acc, red);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int i = 0; i < 7; ++i) partials[blockIdx.x * 7 + i] = acc[i];
    }
  }
}

template <typename T, bool AS, bool RF>
__global__ __launch_bounds__(256) void k_update6(const T* __restrict__ e, T* __restrict__ eps,
                                                 const uint8_t* __restrict__ phase,
                                                 const PhaseCoef<T>* __restrict__ coef, Dims d,
                                                 const T* __restrict__ rf) {
  const long long N = d.N;
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < N; v += (long long)gridDim.x * blockDim.x) {
    const long long vb = zblk(d, v);  // e: the inverse transform output, z-blocked
    if (AS) {
      const PhaseCoef<T> pc = coef[phase[v]];
      T cur[6], dd[6];
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        cur[k] = eps[k * N + v];
        dd[k] = (RF ? e[k * N + vb] + rf[k * N + v] : e[k * N + vb]) - cur[k];
      }
      const T sph = (dd[0] + dd[1] + dd[2]) * T(1.0 / 3.0);
#pragma unroll
      for (int k = 0; k < 3; ++k) eps[k * N + v] = cur[k] + pc.ak * sph + pc.am * (dd[k] - sph);
#pragma unroll
      for (int k = 3; k < 6; ++k) eps[k * N + v] = cur[k] + pc.am * dd[k];
    } else {
#pragma unroll
      for (int k = 0; k < 6; ++k) eps[k * N + v] = RF ? e[k * N + vb] + rf[k * N + v] : e[k * N + vb];
    }
  }
}

template <typename TE>
__global__ __launch_bounds__(256) void k_residual6(const double* __restrict__ e_hi, const TE* __restrict__ eps,
                                                   TE* __restrict__ r, Dims d) {
  const long long N = d.N;
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < N; v += (long long)gridDim.x * blockDim.x) {
    const long long vb = zblk(d, v);
#pragma unroll
    for (int k = 0; k < 6; ++k) r[k * N + v] = TE(e_hi[k * N + vb] - double(eps[k * N + v]));
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_stress(const T* __restrict__ eps, const uint8_t* __restrict__ phase,
                                                const PhaseCoef<T>* __restrict__ coef, T* __restrict__ sigma,
                                                long long N) {
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < N; v += (long long)gridDim.x * blockDim.x) {
    T e[6], s[6];
    load6(eps, N, v, e);
    const PhaseCoef<T> pc = coef[phase[v]];
    iso_apply(pc.lam, pc.mu, e, s);
#pragma unroll
    for (int k = 0; k < 6; ++k) sigma[k * N + v] = s[k];
  }
}

// --------------------------------------------------------------------------
// final reduction: fixed-order sum of per-block partials (deterministic)
// --------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_reduce(const double* __restrict__ partials, int nblocks, int nv,
                                                double* __restrict__ out, const int* __restrict__ active) {
  __shared__ double red[8 * 16];
  const long long smp = active ? active[blockIdx.x] : 0;
  partials += smp * (long long)nblocks * nv;
  out += smp * 8;
  double acc[8];
  reduce_body(partials, nblocks, nv, acc, red);
  if (threadIdx.x == 0)
    for (int i = 0; i < nv && i < 8; ++i) out[i] = acc[i];
}

// --------------------------------------------------------------------------
// launchers
// --------------------------------------------------------------------------

template <typename T>
void Launch<T>::fill_macro(T* eps, long long N, const double* m, hipStream_t s) {
  hipLaunchKernelGGL((k_fill_macro<T>), dim3(grid_for(N)), dim3(kThreads), 0, s, eps, N, T(m[0]), T(m[1]), T(m[2]),
                     T(m[3]), T(m[4]), T(m[5]));
}

template <typename T>
void Launch<T>::convert_to(T* dst, const void* src, int src_is_double, long long n, hipStream_t s) {
  if (src_is_double)
    hipLaunchKernelGGL((k_convert<T, double>), dim3(grid_for(n)), dim3(kThreads), 0, s, dst,
                       static_cast<const double*>(src), n);
  else
    hipLaunchKernelGGL((k_convert<T, float>), dim3(grid_for(n)), dim3(kThreads), 0, s, dst,
                       static_cast<const float*>(src), n);
}

template <typename T>
void Launch<T>::check_phase(const uint8_t* phase, long long N, int n_phases, int* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_check_phase, dim3(grid_for(N)), dim3(kThreads), 0, s, phase, N, n_phases, flag);
}

template <typename T>
int Launch<T>::div(const T* eps, const uint8_t* phase, const PhaseCoef<T>* coef, T* D, const T* Dsig_base,
                   double* partials, Dims d, int op, hipStream_t s, Batch bt, int nsamp) {
  int nb = 0;
  with_tile<T>(d, [&](auto DXC, auto DYC) {
    constexpr int DX = decltype(DXC)::value, DY = decltype(DYC)::value;
    const DivGrid gd = div_grid<DX, DY>(d);
    const dim3 grid(gd.blocks, nsamp);
    nb = gd.blocks;
    if (op == OP_ROT)
      hipLaunchKernelGGL((k_div<DX, DY, T, T, T, OP_ROT>), grid, dim3(DX * DY), 0, s, eps, phase, coef, D,
                         (T*)nullptr, Dsig_base, partials, d, gd.zchunk, bt);
    else
      hipLaunchKernelGGL((k_div<DX, DY, T, T, T, OP_WP>), grid, dim3(DX * DY), 0, s, eps, phase, coef, D,
                         (T*)nullptr, Dsig_base, partials, d, gd.zchunk, bt);
  });
  return nb;
}

template <typename T>
int Launch<T>::update_div(const T* U, const T* eps_in, T* eps_out, const uint8_t* phase, const PhaseCoef<T>* coef,
                          GreenConst<T> g, const T* rfield, T* D, const T* Dsig_base, double* partials, Dims d, int op,
                          int accelerated, hipStream_t s, Batch bt, const GreenConst<T>* gs, int nsamp) {
  // phase constants staged in LDS: a sample's table (batched) or the plan's 256 entries
  const int ncoef = bt.active ? (bt.ncoef < 256 ? bt.ncoef : 256) : 256;
  int nb = 0;
  with_tile<T>(d, [&](auto DXC, auto DYC) {
    constexpr int DX = decltype(DXC)::value, DY = decltype(DYC)::value;
    const DivGrid gd = div_grid<DX, DY>(d);
    const dim3 grid(gd.blocks, nsamp), block(DX * DY);
    nb = gd.blocks;
#define FE_UD(OPV, ASV)                                                                                          \
  do {                                                                                                             \
    if (rfield)                                                                                                    \
      hipLaunchKernelGGL((k_update_div<DX, DY, T, OPV, ASV, true, true>), grid, block, 0, s, U, eps_in, eps_out,   \
                         phase, coef, ncoef, g, rfield, D, Dsig_base, partials, d, gd.zchunk, bt, gs);             \
    else if (eps_out)                                                                                              \
      hipLaunchKernelGGL((k_update_div<DX, DY, T, OPV, ASV, false, true>), grid, block, 0, s, U, eps_in, eps_out,  \
                         phase, coef, ncoef, g, rfield, D, Dsig_base, partials, d, gd.zchunk, bt, gs);             \
    else                                                                                                           \
      hipLaunchKernelGGL((k_update_div<DX, DY, T, OPV, ASV, false, false>), grid, block, 0, s, U, eps_in, eps_out, \
                         phase, coef, ncoef, g, rfield, D, Dsig_base, partials, d, gd.zchunk, bt, gs);             \
  } while (0)
    if (op == OP_ROT) {
      if (accelerated)
        FE_UD(OP_ROT, true);
      else
        FE_UD(OP_ROT, false);
    } else {
      if (accelerated)
        FE_UD(OP_WP, true);
      else
        FE_UD(OP_WP, false);
    }
#undef FE_UD
  });
  return nb;
}

template <typename TS>
int launch_verify_div(const TS* eps, const uint8_t* phase, const PhaseCoef<double>* coef, double* partials, Dims d,
                      int op, hipStream_t s) {
  return launch_div64(eps, phase, coef, nullptr, (TS*)nullptr, partials, d, op, s);
}

template <typename TS>
int launch_div64(const TS* eps, const uint8_t* phase, const PhaseCoef<double>* coef, double* Dtau, TS* Dsig,
                 double* partials, Dims d, int op, hipStream_t s, Batch bt, int nsamp) {
  constexpr int DX = VerifyTile::DX, DY = VerifyTile::DY;
  const DivGrid gd = div_grid<DX, DY>(d);
  const dim3 grid(gd.blocks, nsamp);
  if (op == OP_ROT)
    hipLaunchKernelGGL((k_div<DX, DY, TS, double, double, OP_ROT>), grid, dim3(DX * DY), 0, s, eps, phase, coef, Dtau,
                       Dsig, (const TS*)nullptr, partials, d, gd.zchunk, bt);
  else
    hipLaunchKernelGGL((k_div<DX, DY, TS, double, double, OP_WP>), grid, dim3(DX * DY), 0, s, eps, phase, coef, Dtau,
                       Dsig, (const TS*)nullptr, partials, d, gd.zchunk, bt);
  return gd.blocks;
}

template <typename TE>
void launch_residual(const double* U, const TE* eps, GreenConst<double> g, TE* r, Dims d, int op, hipStream_t s) {
  const dim3 gr(grid_for(d.N, 1 << 20)), bl(kThreads);
  if (op == OP_ROT)
    hipLaunchKernelGGL((k_residual<TE, OP_ROT>), gr, bl, 0, s, U, eps, g, r, d);
  else
    hipLaunchKernelGGL((k_residual<TE, OP_WP>), gr, bl, 0, s, U, eps, g, r, d);
}

template <typename T>
void Launch<T>::axpy(T* y, const T* x, long long n, hipStream_t s) {
  hipLaunchKernelGGL((k_axpy<T>), dim3(grid_for(n, 1 << 20)), dim3(kThreads), 0, s, y, x, n);
}

template <typename T>
int Launch<T>::dot(const T* a, const T* b, long long n, double* partials, hipStream_t s) {
  hipLaunchKernelGGL((k_dot3<T>), dim3(kCgBlocks), dim3(256), 0, s, a, b, n, partials);
  return kCgBlocks;
}

template <typename T>
int Launch<T>::cg_step(T* v, const T* p, T* r, const T* Q, long long n, double* cgs, double* partials,
                       hipStream_t s) {
  hipLaunchKernelGGL((k_cg_step<T>), dim3(kCgBlocks), dim3(256), 0, s, v, p, r, Q, n, cgs, partials);
  return kCgBlocks;
}

template <typename T>
void Launch<T>::cg_dir(T* p, const T* z, long long n, const double* cgs, int first, hipStream_t s) {
  hipLaunchKernelGGL((k_cg_dir<T>), dim3(kCgBlocks), dim3(256), 0, s, p, z, n, cgs, first);
}

void launch_cg_restart(double* cgs, hipStream_t s) { hipLaunchKernelGGL(k_cg_restart, dim3(1), dim3(64), 0, s, cgs); }

template <typename T>
int Launch<T>::cg6_take(const T* Rb, T* Q, const T* x, int negate, Dims d, double lam0, double mu0, double* partials,
                        hipStream_t s) {
  hipLaunchKernelGGL((k_cg6_take<T>), dim3(kCgBlocks), dim3(256), 0, s, Rb, Q, x, negate ? T(-1) : T(1), d, lam0, mu0,
                     partials);
  return kCgBlocks;
}

template <typename T>
int Launch<T>::cg6_step(T* eps, const T* p, T* r, const T* Q, long long N, double lam0, double mu0, double* cgs,
                        double* partials, hipStream_t s) {
  hipLaunchKernelGGL((k_cg6_step<T>), dim3(kCgBlocks), dim3(256), 0, s, eps, p, r, Q, N, lam0, mu0, cgs, partials);
  return kCgBlocks;
}

template <typename T>
void Launch<T>::tau6(const T* eps, const uint8_t* phase, const PhaseCoef<T>* coef, T* out, int write_sigma,
                     double* partials, int nblocks, Dims d, hipStream_t s) {
  hipLaunchKernelGGL((k_tau6<T>), dim3(nblocks), dim3(kThreads), 0, s, eps, phase, coef, out, write_sigma, partials,
                     d);
}

template <typename T>
void Launch<T>::update6(const T* e, T* eps, const uint8_t* phase, const PhaseCoef<T>* coef, Dims d, int accelerated,
                        hipStream_t s, const T* rfield) {
  const dim3 grid(grid_for(d.N, 1 << 20)), block(kThreads);
  if (accelerated) {
    if (rfield)
      hipLaunchKernelGGL((k_update6<T, true, true>), grid, block, 0, s, e, eps, phase, coef, d, rfield);
    else
      hipLaunchKernelGGL((k_update6<T, true, false>), grid, block, 0, s, e, eps, phase, coef, d, rfield);
  } else {
    if (rfield)
      hipLaunchKernelGGL((k_update6<T, false, true>), grid, block, 0, s, e, eps, phase, coef, d, rfield);
    else
      hipLaunchKernelGGL((k_update6<T, false, false>), grid, block, 0, s, e, eps, phase, coef, d, rfield);
  }
}

template <typename TE>
void launch_residual6(const double* e_hi, const TE* eps, TE* r, Dims d, hipStream_t s) {
  hipLaunchKernelGGL((k_residual6<TE>), dim3(grid_for(d.N, 1 << 20)), dim3(kThreads), 0, s, e_hi, eps, r, d);
}

template <typename T>
void Launch<T>::stress(const T* eps, const uint8_t* phase, const PhaseCoef<T>* coef, T* sigma, long long N,
                       hipStream_t s) {
  hipLaunchKernelGGL((k_stress<T>), dim3(grid_for(N, 1 << 20)), dim3(kThreads), 0, s, eps, phase, coef, sigma, N);
}

void launch_reduce(const double* partials, int nblocks, int nv, double* out, hipStream_t s, const int* active,
                   int nsamp) {
  hipLaunchKernelGGL(k_reduce, dim3(nsamp), dim3(256), 0, s, partials, nblocks, nv, out, active);
}

#define FE_INSTANTIATE(T)                                                                                 \
  template void Launch<T>::fill_macro(T*, long long, const double*, hipStream_t);                        \
  template void Launch<T>::convert_to(T*, const void*, int, long long, hipStream_t);                     \
  template void Launch<T>::check_phase(const uint8_t*, long long, int, int*, hipStream_t);               \
  template int Launch<T>::div(const T*, const uint8_t*, const PhaseCoef<T>*, T*, const T*, double*, Dims, int, \
                              hipStream_t, Batch, int);                                                   \
  template void Launch<T>::axpy(T*, const T*, long long, hipStream_t);                                     \
  template int Launch<T>::dot(const T*, const T*, long long, double*, hipStream_t);                        \
  template int Launch<T>::cg_step(T*, const T*, T*, const T*, long long, double*, double*, hipStream_t);    \
  template void Launch<T>::cg_dir(T*, const T*, long long, const double*, int, hipStream_t);               \
  template int Launch<T>::cg6_take(const T*, T*, const T*, int, Dims, double, double, double*, hipStream_t); \
  template int Launch<T>::cg6_step(T*, const T*, T*, const T*, long long, double, double, double*, double*,  \
                                   hipStream_t);                                                              \
  template int Launch<T>::update_div(const T*, const T*, T*, const uint8_t*, const PhaseCoef<T>*, GreenConst<T>, \
                                     const T*, T*, const T*, double*, Dims, int, int, hipStream_t, Batch,         \
                                     const GreenConst<T>*, int);                                                  \
  template void Launch<T>::tau6(const T*, const uint8_t*, const PhaseCoef<T>*, T*, int, double*, int, Dims, \
                                hipStream_t);                                                             \
  template void Launch<T>::update6(const T*, T*, const uint8_t*, const PhaseCoef<T>*, Dims, int, hipStream_t,   \
                                   const T*);                                                                  \
  template void Launch<T>::stress(const T*, const uint8_t*, const PhaseCoef<T>*, T*, long long, hipStream_t);
FE_INSTANTIATE(float)
FE_INSTANTIATE(double)
#undef FE_INSTANTIATE
template int launch_verify_div<float>(const float*, const uint8_t*, const PhaseCoef<double>*, double*, Dims, int,
                                      hipStream_t);
template int launch_verify_div<double>(const double*, const uint8_t*, const PhaseCoef<double>*, double*, Dims, int,
                                       hipStream_t);
template int launch_div64<float>(const float*, const uint8_t*, const PhaseCoef<double>*, double*, float*, double*,
                                 Dims, int, hipStream_t, Batch, int);
template int launch_div64<double>(const double*, const uint8_t*, const PhaseCoef<double>*, double*, double*, double*,
                                  Dims, int, hipStream_t, Batch, int);
template void launch_residual6<float>(const double*, const float*, float*, Dims, hipStream_t);
template void launch_residual6<double>(const double*, const double*, double*, Dims, hipStream_t);
template void launch_residual<float>(const double*, const float*, GreenConst<double>, float*, Dims, int, hipStream_t);
template void launch_residual<double>(const double*, const double*, GreenConst<double>, double*, Dims, int,
                                      hipStream_t);

}  // namespace fe
