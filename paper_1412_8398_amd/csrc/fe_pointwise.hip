// gfx950 kernels of the Lippmann-Schwinger FFT iteration (Willot, arXiv
// 1412.8398).  Equation numbers refer to the paper.
//
// Layouts: real fields are SoA planes [comp][z][y][x] of N = nx*ny*nz values;
// spectra are half spectra along z: [comp][mz][y][x] complex, mz in [0, nz/2].
// Tensor components use Voigt order (11, 22, 33, 23, 13, 12).
#include "fe_green.h"

namespace fe {

// --------------------------------------------------------------------------
// helpers
// --------------------------------------------------------------------------


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
// periodic index for any i >= -n
__device__ __forceinline__ int pmod(int i, int n) { return (i + n) % n; }

// Strain of the iteration from the gradient gr[i][j] = d_i U_j: e = base +
// sym(gr) (base = eps_bar, or the anchor's residual field); DS (eq. (9))
// returns e, AS (eq. (16)) cur + 2 kappa0/(kappa+kappa0) sph(e - cur)
// + 2 mu0/(mu+mu0) dev(e - cur).
template <typename T, bool AS>
__device__ __forceinline__ void strain_update(const T (&gr)[3][3], const T (&base)[6], const T (&cur)[6],
                                              const PhaseCoef<T>& pc, T (&out)[6]) {
  T e[6];
  e[0] = base[0] + gr[0][0];
  e[1] = base[1] + gr[1][1];
  e[2] = base[2] + gr[2][2];
  e[3] = base[3] + T(0.5) * (gr[1][2] + gr[2][1]);
  e[4] = base[4] + T(0.5) * (gr[0][2] + gr[2][0]);
  e[5] = base[5] + T(0.5) * (gr[0][1] + gr[1][0]);
  if (AS) {
    T dd[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) dd[k] = e[k] - cur[k];
    const T sph = (dd[0] + dd[1] + dd[2]) * T(1.0 / 3.0);
#pragma unroll
    for (int k = 0; k < 3; ++k) out[k] = cur[k] + pc.ak * sph + pc.am * (dd[k] - sph);
#pragma unroll
    for (int k = 3; k < 6; ++k) out[k] = cur[k] + pc.am * dd[k];
  } else {
#pragma unroll
    for (int k = 0; k < 6; ++k) out[k] = e[k];
  }
}

// ROT gradient at a voxel from U at its 8 corners, u[a] with a = ax + 2 ay + 4 az:
// d_i U_j = 1/4 sum_a s_i(a) U_j(v + a), s_i(a) = +1 if a_i = 1 else -1 (eq. (37)).
template <typename T>
__device__ __forceinline__ void grad_rot(const T (&u)[8][3], T (&gr)[3][3]) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) gr[i][j] = T(0);
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const T sg[3] = {(a & 1) ? T(1) : T(-1), (a & 2) ? T(1) : T(-1), (a & 4) ? T(1) : T(-1)};
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) gr[i][j] += sg[i] * u[a][j];
  }
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) gr[i][j] *= T(0.25);
}

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

// The corner stencil is separable.  With S_l f(c) = f(c) + f(c - e_l) and
// D_l f(c) = f(c - e_l) - f(c),
//   D_j = 1/4 [ S_z (D_x S_y s_xj + S_x D_y s_yj) + D_z (S_x S_y s_zj) ],
// so a workgroup walks a DX x DY tile of corners along z, loads each voxel
// plane (with a one-voxel halo at -x, -y) once into LDS as tau and sigma, and
// keeps the in-plane combinations P = 1/4 (D_x S_y s_xj + S_x D_y s_yj) and
// Q = 1/4 S_x S_y s_zj of the previous plane in registers:
//   D_j(z) = P(z) + P(z-1) + Q(z-1) - Q(z).
// WP uses the same walk with P = [s_xj(x) - s_xj(x-e_x)] + [s_yj(x) - s_yj(x-e_y)],
// Q = s_zj(x): D_j(z) = P(z) + Q(z) - Q(z-1).
// Corner tile (x by y) of a workgroup, by the type held in LDS.  The -x halo
// voxel of a tile costs a whole 128-byte line per row (and U a second one at
// +x): wide tiles make that a small fraction.  Float: 128 x 8 (1024 threads,
// 94 KiB of LDS); double: 32 x 8 (a double 128 x 8 tile does not fit in
// 160 KiB, and 64 x 8 ran the float64 verification stencil slower).
template <typename T>
struct Tile;
template <>
struct Tile<float> {
  static constexpr int DX = 128, DY = 8;
};
template <>
struct Tile<double> {
  static constexpr int DX = 32, DY = 8;
};

// Workgroup barrier that orders LDS accesses only: global loads issued before
// it stay in flight (they prefetch the next plane).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Optional outputs/inputs (null to skip): Dtau receives the divergence of tau
// (type TD), Dsig the divergence of sigma (type TS), and Dsig_base is added to
// the divergence of sigma before it is squared for eta (the divergence of an
// anchor strain when iterating on a correction).  The strain and phase of the
// next voxel plane are prefetched into registers while the current plane's
// divergence is formed; tau and sigma sit in LDS component-major.
template <typename TS, typename TC, typename TD, int OP>
__global__ __launch_bounds__(Tile<TC>::DX * Tile<TC>::DY) void k_div(const TS* __restrict__ eps, const uint8_t* __restrict__ phase,
                                                 const PhaseCoef<TC>* __restrict__ coef, TD* __restrict__ Dtau,
                                                 TS* __restrict__ Dsig, const TS* __restrict__ Dsig_base,
                                                 double* __restrict__ partials, Dims d, int zchunk, Batch bt) {
  constexpr int DX = Tile<TC>::DX, DY = Tile<TC>::DY;
  constexpr int ER = (DX + 1) * (DY + 1), NT = DX * DY, ES = (ER + NT - 1) / NT;
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
  __shared__ TC st[6][DY + 1][DX + 1];
  __shared__ TC ss[6][DY + 1][DX + 1];
  __shared__ double red[7 * 16];
  const long long N = d.N;
  const int nx = d.nx, ny = d.ny, nz = d.nz;
  const int ntx = (nx + DX - 1) / DX, nty = (ny + DY - 1) / DY;
  const int tile = xcd_block(blockIdx.x, gridDim.x);
  const int bx = tile % ntx;
  const int rest = tile / ntx;
  const int by = rest % nty;
  const int bz = rest / nty;
  const int x0 = bx * DX, y0 = by * DY, z0 = bz * zchunk;
  const int z1 = min(nz, z0 + zchunk);
  const int tx = threadIdx.x % DX, ty = threadIdx.x / DX;
  const int x = x0 + tx, y = y0 + ty;
  const bool own = x < nx && y < ny;
  TS ereg[ES][6];
  int preg[ES];
  auto fetch_e = [&](int zz) {
    const int z = pmod(zz, nz);
#pragma unroll
    for (int q = 0; q < ES; ++q) {
      const int idx = threadIdx.x + q * NT;
      if (idx < ER) {
        const int i = idx % (DX + 1), j = idx / (DX + 1);
        const long long v = ((long long)z * ny + pmod(y0 - 1 + j, ny)) * nx + pmod(x0 - 1 + i, nx);
        preg[q] = phase[v];
#pragma unroll
        for (int k = 0; k < 6; ++k) ereg[q][k] = eps[k * N + v];
      }
    }
  };
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  TC pt[3] = {0, 0, 0}, qt[3] = {0, 0, 0}, ps[3] = {0, 0, 0}, qs[3] = {0, 0, 0};
  fetch_e(z0 - 1);
  for (int zz = z0 - 1; zz < z1; ++zz) {
    const int z = zz < 0 ? zz + nz : zz;
#pragma unroll
    for (int q = 0; q < ES; ++q) {
      const int idx = threadIdx.x + q * NT;
      if (idx >= ER) continue;
      const int i = idx % (DX + 1), j = idx / (DX + 1);
      TC e[6];
#pragma unroll
      for (int k = 0; k < 6; ++k) e[k] = TC(ereg[q][k]);
      const PhaseCoef<TC> pc = coef[preg[q]];
      TC t[6], sg[6];
      iso_apply(pc.dlam, pc.dmu, e, t);
      iso_apply(pc.lam, pc.mu, e, sg);
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        st[k][j][i] = t[k];
        ss[k][j][i] = sg[k];
      }
    }
    if (zz + 1 < z1) fetch_e(zz + 1);  // in flight during this plane's divergence
    lds_barrier();
    // voxel c - a for a in {0,1}^2 in the plane: (tx+1-ax, ty+1-ay)
    TC Pt[3], Qt[3], Ps[3], Qs[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const int cx = voigt_of(0, j), cy = voigt_of(1, j), cz = voigt_of(2, j);
      if (OP == OP_ROT) {
        // f(c), f(c-ex), f(c-ey), f(c-ex-ey)
        const TC ax0 = st[cx][ty + 1][tx + 1], ax1 = st[cx][ty + 1][tx], ax2 = st[cx][ty][tx + 1], ax3 = st[cx][ty][tx];
        const TC ay0 = st[cy][ty + 1][tx + 1], ay1 = st[cy][ty + 1][tx], ay2 = st[cy][ty][tx + 1], ay3 = st[cy][ty][tx];
        const TC az0 = st[cz][ty + 1][tx + 1], az1 = st[cz][ty + 1][tx], az2 = st[cz][ty][tx + 1], az3 = st[cz][ty][tx];
        Pt[j] = TC(0.25) * (((ax1 + ax3) - (ax0 + ax2)) + ((ay2 + ay3) - (ay0 + ay1)));
        Qt[j] = TC(0.25) * ((az0 + az1) + (az2 + az3));
        const TC bx0 = ss[cx][ty + 1][tx + 1], bx1 = ss[cx][ty + 1][tx], bx2 = ss[cx][ty][tx + 1], bx3 = ss[cx][ty][tx];
        const TC by0 = ss[cy][ty + 1][tx + 1], by1 = ss[cy][ty + 1][tx], by2 = ss[cy][ty][tx + 1], by3 = ss[cy][ty][tx];
        const TC bz0 = ss[cz][ty + 1][tx + 1], bz1 = ss[cz][ty + 1][tx], bz2 = ss[cz][ty][tx + 1], bz3 = ss[cz][ty][tx];
        Ps[j] = TC(0.25) * (((bx1 + bx3) - (bx0 + bx2)) + ((by2 + by3) - (by0 + by1)));
        Qs[j] = TC(0.25) * ((bz0 + bz1) + (bz2 + bz3));
      } else {
        Pt[j] = (st[cx][ty + 1][tx + 1] - st[cx][ty + 1][tx]) + (st[cy][ty + 1][tx + 1] - st[cy][ty][tx + 1]);
        Qt[j] = st[cz][ty + 1][tx + 1];
        Ps[j] = (ss[cx][ty + 1][tx + 1] - ss[cx][ty + 1][tx]) + (ss[cy][ty + 1][tx + 1] - ss[cy][ty][tx + 1]);
        Qs[j] = ss[cz][ty + 1][tx + 1];
      }
    }
    if (zz >= z0 && own) {
      const long long c = zidx(d, z, y, x);  // corner arrays: z-blocked transform layout
      TC Dt[3], Ds[3];
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        if (OP == OP_ROT) {
          Dt[j] = (Pt[j] + pt[j]) + (qt[j] - Qt[j]);
          Ds[j] = (Ps[j] + ps[j]) + (qs[j] - Qs[j]);
        } else {
          Dt[j] = Pt[j] + (Qt[j] - qt[j]);
          Ds[j] = Ps[j] + (Qs[j] - qs[j]);
        }
      }
      if (Dtau) {
#pragma unroll
        for (int j = 0; j < 3; ++j) Dtau[j * N + c] = TD(Dt[j]);
      }
      if (Dsig) {
#pragma unroll
        for (int j = 0; j < 3; ++j) Dsig[j * N + c] = TS(Ds[j]);
      }
      double q[3] = {double(Ds[0]), double(Ds[1]), double(Ds[2])};
      if (Dsig_base) {
#pragma unroll
        for (int j = 0; j < 3; ++j) q[j] += double(Dsig_base[j * N + c]);
      }
      acc[0] += q[0] * q[0] + q[1] * q[1] + q[2] * q[2];
#pragma unroll
      for (int k = 0; k < 6; ++k) acc[1 + k] += double(ss[k][ty + 1][tx + 1]);
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      pt[j] = Pt[j];
      qt[j] = Qt[j];
      ps[j] = Ps[j];
      qs[j] = Qs[j];
    }
    lds_barrier();  // st/ss are rewritten by the next plane
  }
  block_sum<7>(acc, red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < 7; ++i) partials[blockIdx.x * 7 + i] = acc[i];
  }
}

// --------------------------------------------------------------------------
// fused strain update and divergence (WP, ROT): from U (the inverse transform
// of iteration k) and eps^k, compute eps^(k+1) and, in the same walk along z,
// the divergences of tau(eps^(k+1)) and sigma(eps^(k+1)) with eta's partial
// sums -- a strain update followed by k_div without writing eps^(k+1)
// and reading it back.  Same tiles, walk and reductions as k_div.  The voxels
// of the -x, -y halo are recomputed (their owner tile writes them), so eps^k
// and eps^(k+1) must be different buffers.
//   U plane z and z+1 in LDS (corners / voxels x0-1 .. x0+DX, y0-1 .. y0+DY),
//   eps^(k+1), tau, sigma of voxel plane z (x0-1 .. x0+DX-1, y0-1 .. y0+DY-1).
// --------------------------------------------------------------------------
template <typename T, int OP, bool AS, bool RF, bool WE>
__global__ __launch_bounds__(Tile<T>::DX * Tile<T>::DY) void k_update_div(const T* __restrict__ U, const T* __restrict__ eps_in,
                                                        T* __restrict__ eps_out, const uint8_t* __restrict__ phase,
                                                        const PhaseCoef<T>* __restrict__ coef, int ncoef,
                                                        GreenConst<T> g, const T* __restrict__ rfield,
                                                        T* __restrict__ Dtau, const T* __restrict__ Dsig_base,
                                                        double* __restrict__ partials, Dims d, int zchunk, Batch bt,
                                                        const GreenConst<T>* __restrict__ gs) {
  constexpr int DX = Tile<T>::DX, DY = Tile<T>::DY;
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
  constexpr int UR = (DX + 2) * (DY + 2), ER = (DX + 1) * (DY + 1), NT = DX * DY;
  constexpr int US = (UR + NT - 1) / NT, ES = (ER + NT - 1) / NT;  // per-thread slots
  __shared__ T su[2][3][DY + 2][DX + 2];  // component-major: consecutive lanes hit consecutive banks
  __shared__ T st[6][DY + 1][DX + 1];
  __shared__ T ss[6][DY + 1][DX + 1];
  __shared__ PhaseCoef<T> sc[256];
  __shared__ double red[7 * 16];
  const int nx = d.nx, ny = d.ny, nz = d.nz;
  const int ntx = (nx + DX - 1) / DX, nty = (ny + DY - 1) / DY;
  const int tile = xcd_block(blockIdx.x, gridDim.x);
  const int bx = tile % ntx;
  const int rest = tile / ntx;
  const int by = rest % nty;
  const int bz = rest / nty;
  const int x0 = bx * DX, y0 = by * DY, z0 = bz * zchunk;
  const int z1 = min(nz, z0 + zchunk);
  const int tx = threadIdx.x % DX, ty = threadIdx.x / DX;
  const int x = x0 + tx, y = y0 + ty;
  const bool own = x < nx && y < ny;
  for (int i = threadIdx.x; i < ncoef; i += NT) sc[i] = coef[i];

  // register prefetch of the next planes: U (corners), eps^k and phase (voxels)
  T ureg[US][3];
  T ereg[ES][6];
  int preg[ES];
  auto fetch_u = [&](int zz) {
    const int z = pmod(zz, nz);
#pragma unroll
    for (int q = 0; q < US; ++q) {
      const int idx = threadIdx.x + q * NT;
      if (idx < UR) {
        const int i = idx % (DX + 2), j = idx / (DX + 2);
        const long long c = zidx(d, z, pmod(y0 - 1 + j, ny), pmod(x0 - 1 + i, nx));  // z-blocked U
#pragma unroll
        for (int k = 0; k < 3; ++k) ureg[q][k] = U[k * N + c];
      }
    }
  };
  auto store_u = [&](int buf) {
#pragma unroll
    for (int q = 0; q < US; ++q) {
      const int idx = threadIdx.x + q * NT;
      if (idx < UR) {
        const int i = idx % (DX + 2), j = idx / (DX + 2);
#pragma unroll
        for (int k = 0; k < 3; ++k) su[buf][k][j][i] = ureg[q][k];
      }
    }
  };
  auto fetch_e = [&](int zz) {
    const int z = pmod(zz, nz);
#pragma unroll
    for (int q = 0; q < ES; ++q) {
      const int idx = threadIdx.x + q * NT;
      if (idx < ER) {
        const int i = idx % (DX + 1), j = idx / (DX + 1);
        const long long v = ((long long)z * ny + pmod(y0 - 1 + j, ny)) * nx + pmod(x0 - 1 + i, nx);
        preg[q] = phase[v];
#pragma unroll
        for (int k = 0; k < 6; ++k) ereg[q][k] = AS ? eps_in[k * N + v] : T(0);
      }
    }
  };

  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  T pt[3] = {0, 0, 0}, qt[3] = {0, 0, 0}, ps[3] = {0, 0, 0}, qs[3] = {0, 0, 0};
  fetch_u(z0 - 1);
  store_u(0);
  fetch_u(z0);
  fetch_e(z0 - 1);
  for (int zz = z0 - 1; zz < z1; ++zz) {
    const int b = (zz - z0 + 1) & 1;  // su[b]: plane zz, su[b ^ 1]: plane zz + 1
    store_u(b ^ 1);
    if (zz + 1 < z1) fetch_u(zz + 2);  // in flight during this plane's update
    lds_barrier();
    const int z = zz < 0 ? zz + nz : zz;
#pragma unroll
    for (int q = 0; q < ES; ++q) {
      const int idx = threadIdx.x + q * NT;
      if (idx >= ER) continue;
      const int i = idx % (DX + 1), j = idx / (DX + 1);
      const int xg = x0 - 1 + i, yg = y0 - 1 + j;
      const long long v = ((long long)z * ny + pmod(yg, ny)) * nx + pmod(xg, nx);
      T gr[3][3];
      if (OP == OP_ROT) {
        T u[8][3];
#pragma unroll
        for (int a = 0; a < 8; ++a)
#pragma unroll
          for (int k = 0; k < 3; ++k) u[a][k] = su[b ^ (a >> 2)][k][j + ((a >> 1) & 1)][i + (a & 1)];
        grad_rot(u, gr);
      } else {
#pragma unroll
        for (int jj = 0; jj < 3; ++jj) {
          const T u0 = su[b][jj][j][i];
          gr[0][jj] = su[b][jj][j][i + 1] - u0;
          gr[1][jj] = su[b][jj][j + 1][i] - u0;
          gr[2][jj] = su[b ^ 1][jj][j][i] - u0;
        }
      }
      T base[6];
#pragma unroll
      for (int k = 0; k < 6; ++k) base[k] = RF ? rfield[k * N + v] : g.macro[k];
      const PhaseCoef<T> pc = sc[preg[q]];
      T e[6];
      strain_update<T, AS>(gr, base, ereg[q], pc, e);
      if (WE && i >= 1 && j >= 1 && xg < nx && yg < ny && zz >= z0)
#pragma unroll
        for (int k = 0; k < 6; ++k) eps_out[k * N + v] = e[k];
      T t[6], sg[6];
      iso_apply(pc.dlam, pc.dmu, e, t);
      iso_apply(pc.lam, pc.mu, e, sg);
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        st[k][j][i] = t[k];
        ss[k][j][i] = sg[k];
      }
    }
    // without the strain write (conjugate gradients) the first sum is U.D at
    // the owned corners: read this corner's U before su[b] is refilled
    T uc[3] = {T(0), T(0), T(0)};
    if (!WE) {
#pragma unroll
      for (int k = 0; k < 3; ++k) uc[k] = su[b][k][ty + 1][tx + 1];
    }
    if (zz + 1 < z1) fetch_e(zz + 1);  // in flight during the divergence and the next store
    lds_barrier();
    T Pt[3], Qt[3], Ps[3], Qs[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const int cx = voigt_of(0, j), cy = voigt_of(1, j), cz = voigt_of(2, j);
      if (OP == OP_ROT) {
        const T ax0 = st[cx][ty + 1][tx + 1], ax1 = st[cx][ty + 1][tx], ax2 = st[cx][ty][tx + 1], ax3 = st[cx][ty][tx];
        const T ay0 = st[cy][ty + 1][tx + 1], ay1 = st[cy][ty + 1][tx], ay2 = st[cy][ty][tx + 1], ay3 = st[cy][ty][tx];
        const T az0 = st[cz][ty + 1][tx + 1], az1 = st[cz][ty + 1][tx], az2 = st[cz][ty][tx + 1], az3 = st[cz][ty][tx];
        Pt[j] = T(0.25) * (((ax1 + ax3) - (ax0 + ax2)) + ((ay2 + ay3) - (ay0 + ay1)));
        Qt[j] = T(0.25) * ((az0 + az1) + (az2 + az3));
        const T bx0 = ss[cx][ty + 1][tx + 1], bx1 = ss[cx][ty + 1][tx], bx2 = ss[cx][ty][tx + 1], bx3 = ss[cx][ty][tx];
        const T by0 = ss[cy][ty + 1][tx + 1], by1 = ss[cy][ty + 1][tx], by2 = ss[cy][ty][tx + 1], by3 = ss[cy][ty][tx];
        const T bz0 = ss[cz][ty + 1][tx + 1], bz1 = ss[cz][ty + 1][tx], bz2 = ss[cz][ty][tx + 1], bz3 = ss[cz][ty][tx];
        Ps[j] = T(0.25) * (((bx1 + bx3) - (bx0 + bx2)) + ((by2 + by3) - (by0 + by1)));
        Qs[j] = T(0.25) * ((bz0 + bz1) + (bz2 + bz3));
      } else {
        Pt[j] = (st[cx][ty + 1][tx + 1] - st[cx][ty + 1][tx]) + (st[cy][ty + 1][tx + 1] - st[cy][ty][tx + 1]);
        Qt[j] = st[cz][ty + 1][tx + 1];
        Ps[j] = (ss[cx][ty + 1][tx + 1] - ss[cx][ty + 1][tx]) + (ss[cy][ty + 1][tx + 1] - ss[cy][ty][tx + 1]);
        Qs[j] = ss[cz][ty + 1][tx + 1];
      }
    }
    if (zz >= z0 && own) {
      const long long c = zidx(d, z, y, x);  // corner arrays: z-blocked transform layout
      T Dt[3], Ds[3];
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        if (OP == OP_ROT) {
          Dt[j] = (Pt[j] + pt[j]) + (qt[j] - Qt[j]);
          Ds[j] = (Ps[j] + ps[j]) + (qs[j] - Qs[j]);
        } else {
          Dt[j] = Pt[j] + (Qt[j] - qt[j]);
          Ds[j] = Ps[j] + (Qs[j] - qs[j]);
        }
      }
#pragma unroll
      for (int j = 0; j < 3; ++j) Dtau[j * N + c] = Dt[j];
      double qd[3] = {double(Ds[0]), double(Ds[1]), double(Ds[2])};
      if (Dsig_base) {
#pragma unroll
        for (int j = 0; j < 3; ++j) qd[j] += double(Dsig_base[j * N + c]);
      }
      if (WE)
        acc[0] += qd[0] * qd[0] + qd[1] * qd[1] + qd[2] * qd[2];
      else
        acc[0] += double(uc[0]) * double(Dt[0]) + double(uc[1]) * double(Dt[1]) + double(uc[2]) * double(Dt[2]);
#pragma unroll
      for (int k = 0; k < 6; ++k) acc[1 + k] += double(ss[k][ty + 1][tx + 1]);
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      pt[j] = Pt[j];
      qt[j] = Qt[j];
      ps[j] = Ps[j];
      qs[j] = Qs[j];
    }
    // st/ss are rewritten after the next step's first barrier, su[b] after this
    // step's second: no third barrier needed
  }
  __syncthreads();
  block_sum<7>(acc, red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < 7; ++i) partials[blockIdx.x * 7 + i] = acc[i];
  }
}

// Tiling of the divergence walk: one corner tile and z chunk per workgroup,
// z cut into chunks of 8 to 64 planes so that a launch has at least about 2M
// threads (several generations of resident workgroups on 256 CUs).
struct DivGrid {
  int blocks, zchunk;
};
template <typename TC>
static DivGrid div_grid(const Dims& d) {
  constexpr int DX = Tile<TC>::DX, DY = Tile<TC>::DY;
  const int ntx = (d.nx + DX - 1) / DX, nty = (d.ny + DY - 1) / DY;
  const int bxy = ntx * nty;
  const int target = (1 << 21) / (DX * DY);
  int nch = (target + bxy - 1) / bxy;
  // chunks of at most 64 planes: neighbouring tiles that start together stay
  // within a few planes of each other, so the halo lines they share are still
  // in L2 when the second one reads them (1024^3: 56 -> 50 B/voxel fetched)
  if (nch < d.nz / 64) nch = d.nz / 64;
  if (nch > kMaxReduceBlocks / bxy) nch = kMaxReduceBlocks / bxy;
  if (nch > d.nz / 8) nch = d.nz / 8;  // chunks of at least 8 planes (one halo plane each)
  if (nch < 1) nch = 1;
  const int zchunk = (d.nz + nch - 1) / nch;
  nch = (d.nz + zchunk - 1) / zchunk;
  return DivGrid{bxy * nch, zchunk};
}

int div_partial_count(Dims d) {
  const int a = div_grid<float>(d).blocks, b = div_grid<double>(d).blocks;
  return a > b ? a : b;
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
  const DivGrid gd = div_grid<T>(d);
  const dim3 grid(gd.blocks, nsamp);
  constexpr int DX = Tile<T>::DX, DY = Tile<T>::DY;
  if (op == OP_ROT)
    hipLaunchKernelGGL((k_div<T, T, T, OP_ROT>), grid, dim3(DX * DY), 0, s, eps, phase, coef, D, (T*)nullptr,
                       Dsig_base, partials, d, gd.zchunk, bt);
  else
    hipLaunchKernelGGL((k_div<T, T, T, OP_WP>), grid, dim3(DX * DY), 0, s, eps, phase, coef, D, (T*)nullptr,
                       Dsig_base, partials, d, gd.zchunk, bt);
  return gd.blocks;
}

template <typename T>
int Launch<T>::update_div(const T* U, const T* eps_in, T* eps_out, const uint8_t* phase, const PhaseCoef<T>* coef,
                          GreenConst<T> g, const T* rfield, T* D, const T* Dsig_base, double* partials, Dims d, int op,
                          int accelerated, hipStream_t s, Batch bt, const GreenConst<T>* gs, int nsamp) {
  const DivGrid gd = div_grid<T>(d);
  const dim3 grid(gd.blocks, nsamp), block(Tile<T>::DX * Tile<T>::DY);
  // phase constants staged in LDS: a sample's table (batched) or the plan's 256 entries
  const int ncoef = bt.active ? (bt.ncoef < 256 ? bt.ncoef : 256) : 256;
#define FE_UD(OPV, ASV)                                                                                          \
  do {                                                                                                             \
    if (rfield)                                                                                                    \
      hipLaunchKernelGGL((k_update_div<T, OPV, ASV, true, true>), grid, block, 0, s, U, eps_in, eps_out, phase,    \
                         coef, ncoef, g, rfield, D, Dsig_base, partials, d, gd.zchunk, bt, gs);                    \
    else if (eps_out)                                                                                              \
      hipLaunchKernelGGL((k_update_div<T, OPV, ASV, false, true>), grid, block, 0, s, U, eps_in, eps_out, phase,   \
                         coef, ncoef, g, rfield, D, Dsig_base, partials, d, gd.zchunk, bt, gs);                    \
    else                                                                                                           \
      hipLaunchKernelGGL((k_update_div<T, OPV, ASV, false, false>), grid, block, 0, s, U, eps_in, eps_out, phase,  \
                         coef, ncoef, g, rfield, D, Dsig_base, partials, d, gd.zchunk, bt, gs);                    \
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
  return gd.blocks;
}

template <typename TS>
int launch_verify_div(const TS* eps, const uint8_t* phase, const PhaseCoef<double>* coef, double* partials, Dims d,
                      int op, hipStream_t s) {
  return launch_div64(eps, phase, coef, nullptr, (TS*)nullptr, partials, d, op, s);
}

template <typename TS>
int launch_div64(const TS* eps, const uint8_t* phase, const PhaseCoef<double>* coef, double* Dtau, TS* Dsig,
                 double* partials, Dims d, int op, hipStream_t s, Batch bt, int nsamp) {
  const DivGrid gd = div_grid<double>(d);
  const dim3 grid(gd.blocks, nsamp);
  constexpr int DX = Tile<double>::DX, DY = Tile<double>::DY;
  if (op == OP_ROT)
    hipLaunchKernelGGL((k_div<TS, double, double, OP_ROT>), grid, dim3(DX * DY), 0, s, eps, phase, coef, Dtau, Dsig,
                       (const TS*)nullptr, partials, d, gd.zchunk, bt);
  else
    hipLaunchKernelGGL((k_div<TS, double, double, OP_WP>), grid, dim3(DX * DY), 0, s, eps, phase, coef, Dtau, Dsig,
                       (const TS*)nullptr, partials, d, gd.zchunk, bt);
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
