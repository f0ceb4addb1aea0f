// gfx950 kernels of the Lippmann-Schwinger FFT iteration (Willot, arXiv
// 1412.8398).  Equation numbers refer to the paper.
//
// Layouts: real fields are SoA planes [comp][z][y][x] of N = nx*ny*nz values;
// spectra are half spectra along z: [comp][mz][y][x] complex, mz in [0, nz/2].
// Tensor components use Voigt order (11, 22, 33, 23, 13, 12).
#include "fe_kernels.h"

namespace fe {

// --------------------------------------------------------------------------
// helpers
// --------------------------------------------------------------------------

// Voigt index of entry (i, j) of a symmetric tensor.
__device__ __forceinline__ int voigt_of(int i, int j) {
  const int s = i + j;
  if (i == j) return i;
  return s == 3 ? 3 : (s == 2 ? 4 : 5);  // (1,2)->3, (0,2)->4, (0,1)->5
}

template <typename T>
__device__ __forceinline__ void load6(const T* __restrict__ f, long long N, long long idx, T (&v)[6]) {
#pragma unroll
  for (int c = 0; c < 6; ++c) v[c] = f[c * N + idx];
}

// sigma = lam tr(eps) I + 2 mu eps  (eq. (2)); same form gives tau with (dlam, dmu).
template <typename T>
__device__ __forceinline__ void iso_apply(T lam, T mu, const T (&e)[6], T (&s)[6]) {
  const T tr = e[0] + e[1] + e[2];
  const T l = lam * tr;
  const T m2 = T(2) * mu;
#pragma unroll
  for (int c = 0; c < 3; ++c) s[c] = l + m2 * e[c];
#pragma unroll
  for (int c = 3; c < 6; ++c) s[c] = m2 * e[c];
}

__device__ __forceinline__ int wrap(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

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

// --------------------------------------------------------------------------
// divergence stencils (displacement form, WP and ROT)
//
// ROT: at corner c (position c - 1/2, i.e. the lower corner of voxel c) the
// divergence of a voxel field s is
//   D_j(c) = 1/4 sum_i [ sum_{a in {0,1}^3, a_i=1} s_ij(c-a) - sum_{a_i=0} s_ij(c-a) ],
// the corner stencil of eq. (38) (up to the factor -1/4); its Fourier symbol
// is conj(k^R) of eq. (36).
// WP: backward differences at voxel x, D_j = sum_i s_ij(x) - s_ij(x - e_i)
// (eq. (23)), symbol -conj(k^W).
// The kernel writes D[tau] and accumulates |D[sigma]|^2 and sum sigma in
// float64 (eq. (43) and eq. (5)).
// --------------------------------------------------------------------------

template <typename TS, typename TC, int OP, bool WRITE_D>
__global__ __launch_bounds__(256) void k_div(const TS* __restrict__ eps, const uint8_t* __restrict__ phase,
                                             const PhaseCoef<TC>* __restrict__ coef, TS* __restrict__ D,
                                             double* __restrict__ partials, Dims d) {
  __shared__ double red[7 * 16];
  const long long N = d.N;
  const int nx = d.nx, ny = d.ny, nz = d.nz;
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < N; c += (long long)gridDim.x * blockDim.x) {
    const int x = (int)(c % nx);
    const int y = (int)((c / nx) % ny);
    const int z = (int)(c / ((long long)nx * ny));
    TC Dt[3] = {0, 0, 0}, Ds[3] = {0, 0, 0};
    if (OP == OP_ROT) {
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        const int ax = a & 1, ay = (a >> 1) & 1, az = (a >> 2) & 1;
        const long long v = ((long long)wrap(z - az, nz) * ny + wrap(y - ay, ny)) * nx + wrap(x - ax, nx);
        TC e[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) e[k] = TC(eps[k * N + v]);
        const PhaseCoef<TC> pc = coef[phase[v]];
        TC t[6], s[6];
        iso_apply(pc.dlam, pc.dmu, e, t);
        iso_apply(pc.lam, pc.mu, e, s);
        const int sg[3] = {ax ? 1 : -1, ay ? 1 : -1, az ? 1 : -1};
#pragma unroll
        for (int j = 0; j < 3; ++j) {
#pragma unroll
          for (int i = 0; i < 3; ++i) {
            const int q = voigt_of(i, j);
            Dt[j] += sg[i] * t[q];
            Ds[j] += sg[i] * s[q];
          }
        }
        if (a == 0) {
#pragma unroll
          for (int k = 0; k < 6; ++k) acc[1 + k] += double(s[k]);
        }
      }
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        Dt[j] *= TC(0.25);
        Ds[j] *= TC(0.25);
      }
    } else {  // OP_WP
      {
        TC e[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) e[k] = TC(eps[k * N + c]);
        const PhaseCoef<TC> pc = coef[phase[c]];
        TC t[6], s[6];
        iso_apply(pc.dlam, pc.dmu, e, t);
        iso_apply(pc.lam, pc.mu, e, s);
#pragma unroll
        for (int j = 0; j < 3; ++j) {
#pragma unroll
          for (int i = 0; i < 3; ++i) {
            Dt[j] += t[voigt_of(i, j)];
            Ds[j] += s[voigt_of(i, j)];
          }
        }
#pragma unroll
        for (int k = 0; k < 6; ++k) acc[1 + k] += double(s[k]);
      }
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const int xm = i == 0 ? wrap(x - 1, nx) : x;
        const int ym = i == 1 ? wrap(y - 1, ny) : y;
        const int zm = i == 2 ? wrap(z - 1, nz) : z;
        const long long v = ((long long)zm * ny + ym) * nx + xm;
        TC e[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) e[k] = TC(eps[k * N + v]);
        const PhaseCoef<TC> pc = coef[phase[v]];
        TC t[6], s[6];
        iso_apply(pc.dlam, pc.dmu, e, t);
        iso_apply(pc.lam, pc.mu, e, s);
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          Dt[j] -= t[voigt_of(i, j)];
          Ds[j] -= s[voigt_of(i, j)];
        }
      }
    }
    if (WRITE_D) {
#pragma unroll
      for (int j = 0; j < 3; ++j) D[j * N + c] = TS(Dt[j]);
    }
    acc[0] += double(Ds[0]) * double(Ds[0]) + double(Ds[1]) * double(Ds[1]) + double(Ds[2]) * double(Ds[2]);
  }
  block_sum<7>(acc, red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < 7; ++i) partials[blockIdx.x * 7 + i] = acc[i];
  }
}

// --------------------------------------------------------------------------
// strain update from the displacement U (WP, ROT)
// ROT: grad at voxel v from its corners v + a: d_i U_j = 1/4 sum_a s_i(a) U_j(v+a),
// s_i(a) = +1 if a_i = 1 else -1 (eq. (37)), symbol k^R.
// WP: forward differences d_i U_j = U_j(v + e_i) - U_j(v) (eq. (23)), symbol k^W.
// e = eps_bar + sym grad U;  DS (eq. (9)): eps <- e;
// AS (eq. (16)): eps <- eps + 2 kappa0/(kappa+kappa0) sph(e - eps) + 2 mu0/(mu+mu0) dev(e - eps).
// --------------------------------------------------------------------------

template <typename T, int OP, bool AS>
__global__ __launch_bounds__(256) void k_grad_update(const T* __restrict__ U, T* __restrict__ eps,
                                                     const uint8_t* __restrict__ phase,
                                                     const PhaseCoef<T>* __restrict__ coef, GreenConst<T> g,
                                                     Dims d) {
  const long long N = d.N;
  const int nx = d.nx, ny = d.ny, nz = d.nz;
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < N; v += (long long)gridDim.x * blockDim.x) {
    const int x = (int)(v % nx);
    const int y = (int)((v / nx) % ny);
    const int z = (int)(v / ((long long)nx * ny));
    T gr[3][3];  // gr[i][j] = d_i U_j
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) gr[i][j] = T(0);
    if (OP == OP_ROT) {
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        const int ax = a & 1, ay = (a >> 1) & 1, az = (a >> 2) & 1;
        const long long c = ((long long)wrap(z + az, nz) * ny + wrap(y + ay, ny)) * nx + wrap(x + ax, nx);
        const T u[3] = {U[c], U[N + c], U[2 * N + c]};
        const T sg[3] = {ax ? T(1) : T(-1), ay ? T(1) : T(-1), az ? T(1) : T(-1)};
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int j = 0; j < 3; ++j) gr[i][j] += sg[i] * u[j];
      }
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) gr[i][j] *= T(0.25);
    } else {
      const T u0[3] = {U[v], U[N + v], U[2 * N + v]};
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const int xp = i == 0 ? wrap(x + 1, nx) : x;
        const int yp = i == 1 ? wrap(y + 1, ny) : y;
        const int zp = i == 2 ? wrap(z + 1, nz) : z;
        const long long c = ((long long)zp * ny + yp) * nx + xp;
#pragma unroll
        for (int j = 0; j < 3; ++j) gr[i][j] = U[j * N + c] - u0[j];
      }
    }
    T e[6];
    e[0] = g.macro[0] + gr[0][0];
    e[1] = g.macro[1] + gr[1][1];
    e[2] = g.macro[2] + gr[2][2];
    e[3] = g.macro[3] + T(0.5) * (gr[1][2] + gr[2][1]);
    e[4] = g.macro[4] + T(0.5) * (gr[0][2] + gr[2][0]);
    e[5] = g.macro[5] + T(0.5) * (gr[0][1] + gr[1][0]);
    if (AS) {
      const PhaseCoef<T> pc = coef[phase[v]];
      T cur[6], dd[6];
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        cur[k] = eps[k * N + v];
        dd[k] = e[k] - cur[k];
      }
      const T sph = (dd[0] + dd[1] + dd[2]) * T(1.0 / 3.0);
#pragma unroll
      for (int k = 0; k < 3; ++k) eps[k * N + v] = cur[k] + pc.ak * sph + pc.am * (dd[k] - sph);
#pragma unroll
      for (int k = 3; k < 6; ++k) eps[k * N + v] = cur[k] + pc.am * dd[k];
    } else {
#pragma unroll
      for (int k = 0; k < 6; ++k) eps[k * N + v] = e[k];
    }
  }
}

// --------------------------------------------------------------------------
// pointwise polarization / stress (6-component form) and update
// --------------------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(256) void k_tau6(const T* __restrict__ eps, const uint8_t* __restrict__ phase,
                                              const PhaseCoef<T>* __restrict__ coef, T* __restrict__ out,
                                              int write_sigma, double* __restrict__ partials, long long N) {
  __shared__ double red[7 * 16];
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < N; v += (long long)gridDim.x * blockDim.x) {
    T e[6];
    load6(eps, N, v, e);
    const PhaseCoef<T> pc = coef[phase[v]];
    T s[6], t[6];
    iso_apply(pc.lam, pc.mu, e, s);
    iso_apply(pc.dlam, pc.dmu, e, t);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      out[k * N + v] = write_sigma ? s[k] : t[k];
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

template <typename T, bool AS>
__global__ __launch_bounds__(256) void k_update6(const T* __restrict__ e, T* __restrict__ eps,
                                                 const uint8_t* __restrict__ phase,
                                                 const PhaseCoef<T>* __restrict__ coef, long long N) {
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < N; v += (long long)gridDim.x * blockDim.x) {
    if (AS) {
      const PhaseCoef<T> pc = coef[phase[v]];
      T cur[6], dd[6];
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        cur[k] = eps[k * N + v];
        dd[k] = e[k * N + v] - cur[k];
      }
      const T sph = (dd[0] + dd[1] + dd[2]) * T(1.0 / 3.0);
#pragma unroll
      for (int k = 0; k < 3; ++k) eps[k * N + v] = cur[k] + pc.ak * sph + pc.am * (dd[k] - sph);
#pragma unroll
      for (int k = 3; k < 6; ++k) eps[k * N + v] = cur[k] + pc.am * dd[k];
    } else {
#pragma unroll
      for (int k = 0; k < 6; ++k) eps[k * N + v] = e[k * N + v];
    }
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
// strided FFT passes
// --------------------------------------------------------------------------

// Forward real-to-complex transform along z.  Two adjacent real x-columns are
// packed as one complex column z = a + i b, transformed, and split with
// A(m) = (Z(m) + conj Z(-m))/2, B(m) = (Z(m) - conj Z(-m))/(2i), m in [0, nz/2].
template <typename T, int NTHR, int CAP>
__global__ __launch_bounds__(NTHR) void k_zr2c(const T* __restrict__ R, cpx<T>* __restrict__ S, Dims d, int ncp_max,
                                               const cpx<T>* __restrict__ tw, uint32_t plan) {
  extern __shared__ unsigned char smem_raw[];
  cpx<T>* tile = reinterpret_cast<cpx<T>*>(smem_raw);
  const int nx = d.nx, ny = d.ny, nz = d.nz, H = d.H;
  const long long N = d.N;
  const int npair = nx / 2;
  const int ntx = (npair + ncp_max - 1) / ncp_max;
  const int xt = blockIdx.x % ntx;
  const int rest = blockIdx.x / ntx;
  const int y = rest % ny;
  const int c = rest / ny;
  const int p0 = xt * ncp_max;
  const int ncp = min(ncp_max, npair - p0);
  const T* src = R + (long long)c * N + (long long)y * nx + 2 * p0;
  for (int idx = threadIdx.x; idx < nz * ncp; idx += NTHR) {
    const int e = idx / ncp, col = idx - e * ncp;
    tile[e * ncp + col] = *reinterpret_cast<const cpx<T>*>(src + (long long)e * ny * nx + 2 * col);
  }
  __syncthreads();
  fft_tile<T, false, NTHR, CAP>(tile, nz, ncp, ncp, 1, tw, plan);
  cpx<T>* dst = S + (long long)c * H * ny * nx + (long long)y * nx + 2 * p0;
  for (int idx = threadIdx.x; idx < H * ncp; idx += NTHR) {
    const int m = idx / ncp, col = idx - m * ncp;
    const cpx<T> Z = tile[m * ncp + col];
    const int mm = m == 0 ? 0 : nz - m;
    const cpx<T> Zm = conj(tile[mm * ncp + col]);
    const cpx<T> A = scale(add(Z, Zm), T(0.5));
    const cpx<T> Dd = sub(Z, Zm);
    const cpx<T> B = mk(T(0.5) * Dd.im, T(-0.5) * Dd.re);
    cpx<T>* o = dst + (long long)m * ny * nx + 2 * col;
    o[0] = A;
    o[1] = B;
  }
}

// Inverse complex-to-real transform along z (unnormalised): rebuilds the full
// spectrum of z = a + i b from the two half spectra A, B using
// Z(m) = A(m) + i B(m) and Z(nz-m) = conj A(m) + i conj B(m).
template <typename T, int NTHR, int CAP>
__global__ __launch_bounds__(NTHR) void k_zc2r(const cpx<T>* __restrict__ S, T* __restrict__ R, Dims d, int ncp_max,
                                               const cpx<T>* __restrict__ tw, uint32_t plan) {
  extern __shared__ unsigned char smem_raw[];
  cpx<T>* tile = reinterpret_cast<cpx<T>*>(smem_raw);
  const int nx = d.nx, ny = d.ny, nz = d.nz, H = d.H;
  const long long N = d.N;
  const int npair = nx / 2;
  const int ntx = (npair + ncp_max - 1) / ncp_max;
  const int xt = blockIdx.x % ntx;
  const int rest = blockIdx.x / ntx;
  const int y = rest % ny;
  const int c = rest / ny;
  const int p0 = xt * ncp_max;
  const int ncp = min(ncp_max, npair - p0);
  const cpx<T>* src = S + (long long)c * H * ny * nx + (long long)y * nx + 2 * p0;
  for (int idx = threadIdx.x; idx < H * ncp; idx += NTHR) {
    const int m = idx / ncp, col = idx - m * ncp;
    const cpx<T>* p = src + (long long)m * ny * nx + 2 * col;
    const cpx<T> A = p[0], B = p[1];
    tile[m * ncp + col] = mk(A.re - B.im, A.im + B.re);
    if (m > 0 && 2 * m < nz) tile[(nz - m) * ncp + col] = mk(A.re + B.im, B.re - A.im);
  }
  __syncthreads();
  fft_tile<T, true, NTHR, CAP>(tile, nz, ncp, ncp, 1, tw, plan);
  T* dst = R + (long long)c * N + (long long)y * nx + 2 * p0;
  for (int idx = threadIdx.x; idx < nz * ncp; idx += NTHR) {
    const int e = idx / ncp, col = idx - e * ncp;
    *reinterpret_cast<cpx<T>*>(dst + (long long)e * ny * nx + 2 * col) = tile[e * ncp + col];
  }
}

// Complex transform along y of the half spectrum, in place.
template <typename T, bool INV, int NTHR, int CAP>
__global__ __launch_bounds__(NTHR) void k_yfft(cpx<T>* __restrict__ S, Dims d, int ncol_max,
                                               const cpx<T>* __restrict__ tw, uint32_t plan) {
  extern __shared__ unsigned char smem_raw[];
  cpx<T>* tile = reinterpret_cast<cpx<T>*>(smem_raw);
  const int nx = d.nx, ny = d.ny, H = d.H;
  const int ntx = (nx + ncol_max - 1) / ncol_max;
  const int xt = blockIdx.x % ntx;
  const int rest = blockIdx.x / ntx;
  const int mz = rest % H;
  const int c = rest / H;
  const int x0 = xt * ncol_max;
  const int nc = min(ncol_max, nx - x0);
  cpx<T>* base = S + (long long)c * H * ny * nx + (long long)mz * ny * nx + x0;
  for (int idx = threadIdx.x; idx < ny * nc; idx += NTHR) {
    const int e = idx / nc, col = idx - e * nc;
    tile[e * nc + col] = base[(long long)e * nx + col];
  }
  __syncthreads();
  fft_tile<T, INV, NTHR, CAP>(tile, ny, nc, nc, 1, tw, plan);
  for (int idx = threadIdx.x; idx < ny * nc; idx += NTHR) {
    const int e = idx / nc, col = idx - e * nc;
    base[(long long)e * nx + col] = tile[e * nc + col];
  }
}

// --------------------------------------------------------------------------
// x pass with the Green operator (contiguous lines)
// --------------------------------------------------------------------------

// Displacement form: given b-like D(q) (3 comps) return u(q) = -+ A^-1 b / N.
// ROT: k^R = 2i exp(i phi) t with t_a = sin(q_a/2) prod_{b!=a} cos(q_b/2) (eq. (36)),
//      A = 4 (lam0+mu0) t t^T + 4 mu0 |t|^2 I, b = D (corner stencil symbol conj k^R),
//      u = -A^-1 b = -(b - cr t (t.b)/|t|^2) / (4 mu0 |t|^2).  |t| = 0 at q = 0 and where
//      two q_i equal pi: u = 0 there (eq. (41)).
// WP:  k = exp(iq) - 1, b = -D (backward-difference symbol is -conj k), u = A^-1 D with
//      A = lam0 conj(k) k^T + mu0 k conj(k)^T + mu0 |k|^2 I solved by the Woodbury
//      identity over the rank-2 part (eq. (19)).
template <typename T>
__device__ __forceinline__ void woodbury_solve(const cpx<T> (&k)[3], const cpx<T> (&b)[3], T lam0, T mu0,
                                               cpx<T> (&x)[3]) {
  // A = D I + lam0 conj(k) k^T + mu0 k conj(k)^T, D = mu0 n2
  const T n2 = norm2(k[0]) + norm2(k[1]) + norm2(k[2]);
  const cpx<T> s = add(add(mul(k[0], k[0]), mul(k[1], k[1])), mul(k[2], k[2]));  // k.k
  const cpx<T> p = add(add(mul(k[0], b[0]), mul(k[1], b[1])), mul(k[2], b[2]));  // k^T b
  const cpx<T> r = add(add(mul(conj(k[0]), b[0]), mul(conj(k[1]), b[1])), mul(conj(k[2]), b[2]));  // k^H b
  const T Dg = mu0 * n2;
  // M = [[(lam0+mu0) n2, lam0 s], [mu0 conj s, 2 mu0 n2]], rhs = [lam0 p, mu0 r]
  const T det = T(2) * mu0 * (lam0 + mu0) * n2 * n2 - lam0 * mu0 * norm2(s);
  const T idet = T(1) / det;
  const cpx<T> y1 = scale(sub(scale(p, T(2) * mu0 * n2 * lam0), scale(mul(s, r), lam0 * mu0)), idet);
  const cpx<T> y2 = scale(sub(scale(r, (lam0 + mu0) * n2 * mu0), scale(mul(conj(s), p), mu0 * lam0)), idet);
  const T iD = T(1) / Dg;
#pragma unroll
  for (int a = 0; a < 3; ++a) x[a] = scale(sub(sub(b[a], mul(conj(k[a]), y1)), mul(k[a], y2)), iD);
}

template <typename T, int OP>
__device__ __forceinline__ void wave_k(const WaveTables<T>& wt, int mx, int my, int mz, cpx<T> (&k)[3]) {
  const T ax = wt.x[2 * mx], bx = wt.x[2 * mx + 1];
  const T ay = wt.y[2 * my], by = wt.y[2 * my + 1];
  const T az = wt.z[2 * mz], bz = wt.z[2 * mz + 1];
  if (OP == OP_WP) {
    k[0] = mk(ax, bx);
    k[1] = mk(ay, by);
    k[2] = mk(az, bz);
  } else if (OP == OP_MS) {
    k[0] = mk(T(0), ax);
    k[1] = mk(T(0), ay);
    k[2] = mk(T(0), az);
  } else {  // ROT: 2 i exp(i phi) t, exp(i phi) = prod (cos + i sin) of half angles
    const T t0 = ax * by * bz, t1 = ay * bx * bz, t2 = az * bx * by;
    const cpx<T> ph = mul(mul(mk(bx, ax), mk(by, ay)), mk(bz, az));
    const cpx<T> f = mk(-T(2) * ph.im, T(2) * ph.re);  // 2 i ph
    k[0] = scale(f, t0);
    k[1] = scale(f, t1);
    k[2] = scale(f, t2);
  }
}

template <typename T, int OP, int NTHR, int CAP>
__global__ __launch_bounds__(NTHR) void k_xgreen3(cpx<T>* __restrict__ S, Dims d, int nl_max,
                                                  const cpx<T>* __restrict__ tw, uint32_t plan, WaveTables<T> wt,
                                                  GreenConst<T> g) {
  extern __shared__ unsigned char smem_raw[];
  cpx<T>* tile = reinterpret_cast<cpx<T>*>(smem_raw);
  const int nx = d.nx, ny = d.ny, H = d.H;
  const long long cs = (long long)H * ny * nx;
  const int nlines = H * ny;
  const int line0 = blockIdx.x * nl_max;
  const int nl = min(nl_max, nlines - line0);
  const int ncol = 3 * nl;
  for (int idx = threadIdx.x; idx < ncol * nx; idx += NTHR) {
    const int e = idx % nx, cl = idx / nx;
    const int c = cl / nl, l = cl - c * nl;
    tile[e * ncol + cl] = S[c * cs + (long long)(line0 + l) * nx + e];
  }
  __syncthreads();
  fft_tile<T, false, NTHR, CAP>(tile, nx, ncol, ncol, 1, tw, plan);
  for (int idx = threadIdx.x; idx < nl * nx; idx += NTHR) {
    const int e = idx % nx, l = idx / nx;
    const int line = line0 + l;
    const int mz = line / ny, my = line - mz * ny, mx = e;
    cpx<T> b[3], u[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) b[c] = tile[e * ncol + c * nl + l];
    if (OP == OP_ROT) {
      const T ax = wt.x[2 * mx], bx = wt.x[2 * mx + 1];
      const T ay = wt.y[2 * my], by = wt.y[2 * my + 1];
      const T az = wt.z[2 * mz], bz = wt.z[2 * mz + 1];
      const T t[3] = {ax * by * bz, ay * bx * bz, az * bx * by};
      const T tt = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
      if (tt > T(0)) {
        const cpx<T> tb = add(add(scale(b[0], t[0]), scale(b[1], t[1])), scale(b[2], t[2]));
        const T f = -g.inv_n / (T(4) * g.mu0 * tt);
        const T h = g.cr / tt;
#pragma unroll
        for (int a = 0; a < 3; ++a) u[a] = scale(sub(b[a], scale(tb, h * t[a])), f);
      } else {
#pragma unroll
        for (int a = 0; a < 3; ++a) u[a] = mk(T(0), T(0));
      }
    } else {  // OP_WP
      cpx<T> k[3];
      wave_k<T, OP_WP>(wt, mx, my, mz, k);
      if (mx == 0 && my == 0 && mz == 0) {
#pragma unroll
        for (int a = 0; a < 3; ++a) u[a] = mk(T(0), T(0));
      } else {
        woodbury_solve(k, b, g.lam0, g.mu0, u);
#pragma unroll
        for (int a = 0; a < 3; ++a) u[a] = scale(u[a], g.inv_n);
      }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) tile[e * ncol + c * nl + l] = u[c];
  }
  __syncthreads();
  fft_tile<T, true, NTHR, CAP>(tile, nx, ncol, ncol, 1, tw, plan);
  for (int idx = threadIdx.x; idx < ncol * nx; idx += NTHR) {
    const int e = idx % nx, cl = idx / nx;
    const int c = cl / nl, l = cl - c * nl;
    S[c * cs + (long long)(line0 + l) * nx + e] = tile[e * ncol + cl];
  }
}

// Six-component Green operator (any operator): for an ordinary q,
// b_j = sum_i conj(k_i) tau_ij, u = -A^-1 b, eps_ij = (k_i u_j + k_j u_i)/2 (eq. (19));
// q = 0: eps = eps_bar (mean, eq. (6)); MS with some q_i = pi: eps = -(C0)^-1 tau (eq. (14));
// ROT where two q_i equal pi: 0 (eq. (41)).  Results carry the 1/N of eq. (10).
template <typename T, int OP, int NTHR, int CAP>
__global__ __launch_bounds__(NTHR) void k_xgreen6(cpx<T>* __restrict__ S, Dims d, int nl_max,
                                                  const cpx<T>* __restrict__ tw, uint32_t plan, WaveTables<T> wt,
                                                  GreenConst<T> g) {
  extern __shared__ unsigned char smem_raw[];
  cpx<T>* tile = reinterpret_cast<cpx<T>*>(smem_raw);
  const int nx = d.nx, ny = d.ny, nz = d.nz, H = d.H;
  const long long cs = (long long)H * ny * nx;
  const int nlines = H * ny;
  const int line0 = blockIdx.x * nl_max;
  const int nl = min(nl_max, nlines - line0);
  const int ncol = 6 * nl;
  for (int idx = threadIdx.x; idx < ncol * nx; idx += NTHR) {
    const int e = idx % nx, cl = idx / nx;
    const int c = cl / nl, l = cl - c * nl;
    tile[e * ncol + cl] = S[c * cs + (long long)(line0 + l) * nx + e];
  }
  __syncthreads();
  fft_tile<T, false, NTHR, CAP>(tile, nx, ncol, ncol, 1, tw, plan);
  for (int idx = threadIdx.x; idx < nl * nx; idx += NTHR) {
    const int e = idx % nx, l = idx / nx;
    const int line = line0 + l;
    const int mz = line / ny, my = line - mz * ny, mx = e;
    cpx<T> tv[6], ev[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) tv[c] = tile[e * ncol + c * nl + l];
    if (mx == 0 && my == 0 && mz == 0) {
#pragma unroll
      for (int c = 0; c < 6; ++c) ev[c] = mk(g.macro[c], T(0));
    } else {
      bool nyq_ms = false;
      if (OP == OP_MS) nyq_ms = (wt.x[2 * mx + 1] != T(0)) || (wt.y[2 * my + 1] != T(0)) || (wt.z[2 * mz + 1] != T(0));
      if (nyq_ms) {
        const cpx<T> tr = add(add(tv[0], tv[1]), tv[2]);
#pragma unroll
        for (int c = 0; c < 6; ++c) ev[c] = scale(tv[c], -g.s1 * g.inv_n);
#pragma unroll
        for (int c = 0; c < 3; ++c) ev[c] = add(ev[c], scale(tr, g.s2 * g.inv_n));
      } else {
        cpx<T> k[3];
        wave_k<T, OP>(wt, mx, my, mz, k);
        const T n2 = norm2(k[0]) + norm2(k[1]) + norm2(k[2]);
        if (n2 > T(0)) {
          cpx<T> b[3], u[3];
#pragma unroll
          for (int j = 0; j < 3; ++j) {
            cpx<T> acc = mk(T(0), T(0));
#pragma unroll
            for (int i = 0; i < 3; ++i) acc = add(acc, mul(conj(k[i]), tv[voigt_of(i, j)]));
            b[j] = acc;
          }
          woodbury_solve(k, b, g.lam0, g.mu0, u);
          // eps = sym(k (x) u) with u = -A^-1 b, times 1/N
          const T f = -g.inv_n;
          ev[0] = scale(mul(k[0], u[0]), f);
          ev[1] = scale(mul(k[1], u[1]), f);
          ev[2] = scale(mul(k[2], u[2]), f);
          ev[3] = scale(add(mul(k[1], u[2]), mul(k[2], u[1])), T(0.5) * f);
          ev[4] = scale(add(mul(k[0], u[2]), mul(k[2], u[0])), T(0.5) * f);
          ev[5] = scale(add(mul(k[0], u[1]), mul(k[1], u[0])), T(0.5) * f);
        } else {
#pragma unroll
          for (int c = 0; c < 6; ++c) ev[c] = mk(T(0), T(0));
        }
      }
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) tile[e * ncol + c * nl + l] = ev[c];
  }
  __syncthreads();
  fft_tile<T, true, NTHR, CAP>(tile, nx, ncol, ncol, 1, tw, plan);
  for (int idx = threadIdx.x; idx < ncol * nx; idx += NTHR) {
    const int e = idx % nx, cl = idx / nx;
    const int c = cl / nl, l = cl - c * nl;
    S[c * cs + (long long)(line0 + l) * nx + e] = tile[e * ncol + cl];
  }
}

// Spectral equilibrium norm (eq. (43)) from the half spectrum of sigma: each
// stored q with 0 < mz < nz/2 also stands for its mirror q' = -q (mod grid),
// whose coefficient is conj sigma(q) and whose wave vector is read from the
// tables at the mirror indices.  Accumulates sum |conj(k).sigma|^2 in float64.
template <typename T, int OP, int NTHR, int CAP>
__global__ __launch_bounds__(NTHR) void k_xeta6(const cpx<T>* __restrict__ S, Dims d, int nl_max,
                                                const cpx<T>* __restrict__ tw, uint32_t plan, WaveTables<T> wt,
                                                double* __restrict__ partials) {
  extern __shared__ unsigned char smem_raw[];
  __shared__ double red[16];
  cpx<T>* tile = reinterpret_cast<cpx<T>*>(smem_raw);
  const int nx = d.nx, ny = d.ny, nz = d.nz, H = d.H;
  const long long cs = (long long)H * ny * nx;
  const int nlines = H * ny;
  const int line0 = blockIdx.x * nl_max;
  const int nl = min(nl_max, nlines - line0);
  const int ncol = 6 * nl;
  for (int idx = threadIdx.x; idx < ncol * nx; idx += NTHR) {
    const int e = idx % nx, cl = idx / nx;
    const int c = cl / nl, l = cl - c * nl;
    tile[e * ncol + cl] = S[c * cs + (long long)(line0 + l) * nx + e];
  }
  __syncthreads();
  fft_tile<T, false, NTHR, CAP>(tile, nx, ncol, ncol, 1, tw, plan);
  double acc[1] = {0.0};
  for (int idx = threadIdx.x; idx < nl * nx; idx += NTHR) {
    const int e = idx % nx, l = idx / nx;
    const int line = line0 + l;
    const int mz = line / ny, my = line - mz * ny, mx = e;
    cpx<T> sv[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) sv[c] = tile[e * ncol + c * nl + l];
    cpx<T> k[3];
    wave_k<T, OP>(wt, mx, my, mz, k);
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      cpx<T> a = mk(T(0), T(0));
#pragma unroll
      for (int i = 0; i < 3; ++i) a = add(a, mul(conj(k[i]), sv[voigt_of(i, j)]));
      s += double(a.re) * double(a.re) + double(a.im) * double(a.im);
    }
    if (mz > 0 && 2 * mz < nz) {
      const int qx = mx == 0 ? 0 : nx - mx, qy = my == 0 ? 0 : ny - my, qz = nz - mz;
      wave_k<T, OP>(wt, qx, qy, qz, k);
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        cpx<T> a = mk(T(0), T(0));
#pragma unroll
        for (int i = 0; i < 3; ++i) a = add(a, mul(conj(k[i]), conj(sv[voigt_of(i, j)])));
        s += double(a.re) * double(a.re) + double(a.im) * double(a.im);
      }
    }
    acc[0] += s;
  }
  block_sum<1>(acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = acc[0];
}

// --------------------------------------------------------------------------
// final reduction: fixed-order sum of per-block partials (deterministic)
// --------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_reduce(const double* __restrict__ partials, int nblocks, int nv,
                                                double* __restrict__ out) {
  __shared__ double red[8 * 16];
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x)
    for (int i = 0; i < nv && i < 8; ++i) acc[i] += partials[(long long)b * nv + i];
  block_sum<8>(acc, red);
  if (threadIdx.x == 0)
    for (int i = 0; i < nv && i < 8; ++i) out[i] = acc[i];
}

// --------------------------------------------------------------------------
// launchers
// --------------------------------------------------------------------------

template <typename T>
static int cols_for(int n, int avail, int cap) {
  int c = cap / n;
  if (c > avail) c = avail;
  if (c >= 16) c &= ~7;
  if (c < 1) c = 1;
  return c;
}

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
void Launch<T>::div(const T* eps, const uint8_t* phase, const PhaseCoef<T>* coef, T* D, double* partials,
                    int nblocks, Dims d, int op, hipStream_t s) {
  if (op == OP_ROT)
    hipLaunchKernelGGL((k_div<T, T, OP_ROT, true>), dim3(nblocks), dim3(kThreads), 0, s, eps, phase, coef, D,
                       partials, d);
  else
    hipLaunchKernelGGL((k_div<T, T, OP_WP, true>), dim3(nblocks), dim3(kThreads), 0, s, eps, phase, coef, D,
                       partials, d);
}

template <typename TS>
void launch_verify_div(const TS* eps, const uint8_t* phase, const PhaseCoef<double>* coef, double* partials,
                       int nblocks, Dims d, int op, hipStream_t s) {
  if (op == OP_ROT)
    hipLaunchKernelGGL((k_div<TS, double, OP_ROT, false>), dim3(nblocks), dim3(kThreads), 0, s, eps, phase, coef,
                       (TS*)nullptr, partials, d);
  else
    hipLaunchKernelGGL((k_div<TS, double, OP_WP, false>), dim3(nblocks), dim3(kThreads), 0, s, eps, phase, coef,
                       (TS*)nullptr, partials, d);
}

template <typename T>
void Launch<T>::grad_update(const T* U, T* eps, const uint8_t* phase, const PhaseCoef<T>* coef, GreenConst<T> g,
                            Dims d, int op, int accelerated, hipStream_t s) {
  const dim3 gr(grid_for(d.N, 1 << 20)), bl(kThreads);
  if (op == OP_ROT) {
    if (accelerated)
      hipLaunchKernelGGL((k_grad_update<T, OP_ROT, true>), gr, bl, 0, s, U, eps, phase, coef, g, d);
    else
      hipLaunchKernelGGL((k_grad_update<T, OP_ROT, false>), gr, bl, 0, s, U, eps, phase, coef, g, d);
  } else {
    if (accelerated)
      hipLaunchKernelGGL((k_grad_update<T, OP_WP, true>), gr, bl, 0, s, U, eps, phase, coef, g, d);
    else
      hipLaunchKernelGGL((k_grad_update<T, OP_WP, false>), gr, bl, 0, s, U, eps, phase, coef, g, d);
  }
}

template <typename T>
void Launch<T>::xgreen3(cpx<T>* S, Dims d, const cpx<T>* twx, uint32_t planx, WaveTables<T> wt, GreenConst<T> g,
                        int op, hipStream_t s) {
  constexpr int CAP = TileCap<T>::CAP;
  int nl = CAP / (3 * d.nx);
  if (nl < 1) nl = 1;
  const int nlines = d.H * d.ny;
  if (nl > nlines) nl = nlines;
  const int nblk = (nlines + nl - 1) / nl;
  const size_t lds = (size_t)3 * nl * d.nx * sizeof(cpx<T>);
  if (op == OP_ROT)
    hipLaunchKernelGGL((k_xgreen3<T, OP_ROT, kThreads, CAP>), dim3(nblk), dim3(kThreads), lds, s, S, d, nl, twx,
                       planx, wt, g);
  else
    hipLaunchKernelGGL((k_xgreen3<T, OP_WP, kThreads, CAP>), dim3(nblk), dim3(kThreads), lds, s, S, d, nl, twx,
                       planx, wt, g);
}

template <typename T>
void Launch<T>::tau6(const T* eps, const uint8_t* phase, const PhaseCoef<T>* coef, T* out, int write_sigma,
                     double* partials, int nblocks, Dims d, hipStream_t s) {
  hipLaunchKernelGGL((k_tau6<T>), dim3(nblocks), dim3(kThreads), 0, s, eps, phase, coef, out, write_sigma, partials,
                     d.N);
}

template <typename T>
void Launch<T>::xgreen6(cpx<T>* S, Dims d, const cpx<T>* twx, uint32_t planx, WaveTables<T> wt, GreenConst<T> g,
                        int op, hipStream_t s) {
  constexpr int CAP = TileCap<T>::CAP6;
  int nl = CAP / (6 * d.nx);
  if (nl < 1) nl = 1;
  const int nlines = d.H * d.ny;
  if (nl > nlines) nl = nlines;
  const int nblk = (nlines + nl - 1) / nl;
  const size_t lds = (size_t)6 * nl * d.nx * sizeof(cpx<T>);
  switch (op) {
    case OP_MS:
      hipLaunchKernelGGL((k_xgreen6<T, OP_MS, kThreads, CAP>), dim3(nblk), dim3(kThreads), lds, s, S, d, nl, twx,
                         planx, wt, g);
      break;
    case OP_WP:
      hipLaunchKernelGGL((k_xgreen6<T, OP_WP, kThreads, CAP>), dim3(nblk), dim3(kThreads), lds, s, S, d, nl, twx,
                         planx, wt, g);
      break;
    default:
      hipLaunchKernelGGL((k_xgreen6<T, OP_ROT, kThreads, CAP>), dim3(nblk), dim3(kThreads), lds, s, S, d, nl, twx,
                         planx, wt, g);
      break;
  }
}

template <typename T>
void Launch<T>::xeta6(const cpx<T>* S, Dims d, const cpx<T>* twx, uint32_t planx, WaveTables<T> wt,
                      double* partials, int nblocks_unused, int op, hipStream_t s) {
  (void)nblocks_unused;
  constexpr int CAP = TileCap<T>::CAP6;
  int nl = CAP / (6 * d.nx);
  if (nl < 1) nl = 1;
  const int nlines = d.H * d.ny;
  if (nl > nlines) nl = nlines;
  const int nblk = (nlines + nl - 1) / nl;
  const size_t lds = (size_t)6 * nl * d.nx * sizeof(cpx<T>);
  switch (op) {
    case OP_MS:
      hipLaunchKernelGGL((k_xeta6<T, OP_MS, kThreads, CAP>), dim3(nblk), dim3(kThreads), lds, s, S, d, nl, twx,
                         planx, wt, partials);
      break;
    case OP_WP:
      hipLaunchKernelGGL((k_xeta6<T, OP_WP, kThreads, CAP>), dim3(nblk), dim3(kThreads), lds, s, S, d, nl, twx,
                         planx, wt, partials);
      break;
    default:
      hipLaunchKernelGGL((k_xeta6<T, OP_ROT, kThreads, CAP>), dim3(nblk), dim3(kThreads), lds, s, S, d, nl, twx,
                         planx, wt, partials);
      break;
  }
}

template <typename T>
void Launch<T>::update6(const T* e, T* eps, const uint8_t* phase, const PhaseCoef<T>* coef, Dims d, int accelerated,
                        hipStream_t s) {
  if (accelerated)
    hipLaunchKernelGGL((k_update6<T, true>), dim3(grid_for(d.N, 1 << 20)), dim3(kThreads), 0, s, e, eps, phase, coef,
                       d.N);
  else
    hipLaunchKernelGGL((k_update6<T, false>), dim3(grid_for(d.N, 1 << 20)), dim3(kThreads), 0, s, e, eps, phase,
                       coef, d.N);
}

template <typename T>
void Launch<T>::zr2c(const T* R, cpx<T>* S, int ncomp, Dims d, const cpx<T>* twz, uint32_t planz, hipStream_t s) {
  constexpr int CAP = TileCap<T>::CAP;
  const int ncp = cols_for<T>(d.nz, d.nx / 2, CAP);
  const int ntx = (d.nx / 2 + ncp - 1) / ncp;
  const size_t lds = (size_t)ncp * d.nz * sizeof(cpx<T>);
  hipLaunchKernelGGL((k_zr2c<T, kThreads, CAP>), dim3(ntx * d.ny * ncomp), dim3(kThreads), lds, s, R, S, d, ncp, twz,
                     planz);
}

template <typename T>
void Launch<T>::zc2r(const cpx<T>* S, T* R, int ncomp, Dims d, const cpx<T>* twz, uint32_t planz, hipStream_t s) {
  constexpr int CAP = TileCap<T>::CAP;
  const int ncp = cols_for<T>(d.nz, d.nx / 2, CAP);
  const int ntx = (d.nx / 2 + ncp - 1) / ncp;
  const size_t lds = (size_t)ncp * d.nz * sizeof(cpx<T>);
  hipLaunchKernelGGL((k_zc2r<T, kThreads, CAP>), dim3(ntx * d.ny * ncomp), dim3(kThreads), lds, s, S, R, d, ncp, twz,
                     planz);
}

template <typename T>
void Launch<T>::yfft(cpx<T>* S, int ncomp, Dims d, const cpx<T>* twy, uint32_t plany, int inverse, hipStream_t s) {
  constexpr int CAP = TileCap<T>::CAP;
  const int nc = cols_for<T>(d.ny, d.nx, CAP);
  const int ntx = (d.nx + nc - 1) / nc;
  const size_t lds = (size_t)nc * d.ny * sizeof(cpx<T>);
  const dim3 gr(ntx * d.H * ncomp);
  if (inverse)
    hipLaunchKernelGGL((k_yfft<T, true, kThreads, CAP>), gr, dim3(kThreads), lds, s, S, d, nc, twy, plany);
  else
    hipLaunchKernelGGL((k_yfft<T, false, kThreads, CAP>), gr, dim3(kThreads), lds, s, S, d, nc, twy, plany);
}

template <typename T>
void Launch<T>::stress(const T* eps, const uint8_t* phase, const PhaseCoef<T>* coef, T* sigma, long long N,
                       hipStream_t s) {
  hipLaunchKernelGGL((k_stress<T>), dim3(grid_for(N, 1 << 20)), dim3(kThreads), 0, s, eps, phase, coef, sigma, N);
}

template <typename T>
int Launch<T>::set_kernel_attributes() {
  constexpr int CAP = TileCap<T>::CAP;
  constexpr int CAP6 = TileCap<T>::CAP6;
  const int l1 = CAP * (int)sizeof(cpx<T>);
  const int l6 = CAP6 * (int)sizeof(cpx<T>);
  int bad = 0;
  bad |= hipFuncSetAttribute((const void*)k_zr2c<T, kThreads, CAP>, hipFuncAttributeMaxDynamicSharedMemorySize, l1);
  bad |= hipFuncSetAttribute((const void*)k_zc2r<T, kThreads, CAP>, hipFuncAttributeMaxDynamicSharedMemorySize, l1);
  bad |= hipFuncSetAttribute((const void*)k_yfft<T, false, kThreads, CAP>, hipFuncAttributeMaxDynamicSharedMemorySize, l1);
  bad |= hipFuncSetAttribute((const void*)k_yfft<T, true, kThreads, CAP>, hipFuncAttributeMaxDynamicSharedMemorySize, l1);
  bad |= hipFuncSetAttribute((const void*)k_xgreen3<T, OP_ROT, kThreads, CAP>, hipFuncAttributeMaxDynamicSharedMemorySize, l1);
  bad |= hipFuncSetAttribute((const void*)k_xgreen3<T, OP_WP, kThreads, CAP>, hipFuncAttributeMaxDynamicSharedMemorySize, l1);
  bad |= hipFuncSetAttribute((const void*)k_xgreen6<T, OP_MS, kThreads, CAP6>, hipFuncAttributeMaxDynamicSharedMemorySize, l6);
  bad |= hipFuncSetAttribute((const void*)k_xgreen6<T, OP_WP, kThreads, CAP6>, hipFuncAttributeMaxDynamicSharedMemorySize, l6);
  bad |= hipFuncSetAttribute((const void*)k_xgreen6<T, OP_ROT, kThreads, CAP6>, hipFuncAttributeMaxDynamicSharedMemorySize, l6);
  bad |= hipFuncSetAttribute((const void*)k_xeta6<T, OP_MS, kThreads, CAP6>, hipFuncAttributeMaxDynamicSharedMemorySize, l6);
  bad |= hipFuncSetAttribute((const void*)k_xeta6<T, OP_WP, kThreads, CAP6>, hipFuncAttributeMaxDynamicSharedMemorySize, l6);
  bad |= hipFuncSetAttribute((const void*)k_xeta6<T, OP_ROT, kThreads, CAP6>, hipFuncAttributeMaxDynamicSharedMemorySize, l6);
  return bad;
}

void launch_reduce(const double* partials, int nblocks, int nv, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(256), 0, s, partials, nblocks, nv, out);
}

template struct Launch<float>;
template struct Launch<double>;
template void launch_verify_div<float>(const float*, const uint8_t*, const PhaseCoef<double>*, double*, int, Dims, int,
                                       hipStream_t);
template void launch_verify_div<double>(const double*, const uint8_t*, const PhaseCoef<double>*, double*, int, Dims,
                                        int, hipStream_t);

}  // namespace fe
