// Divergence stencils and the fused strain update of the displacement form
// (WP, ROT): workgroup bodies shared by the per-pass kernels
// (fe_pointwise.hip) and the persistent batched kernel (fe_batch.hip), so
// both compute the same values in the same order.
#pragma once

#include "fe_green.h"

namespace fe {

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
// 94 KiB of LDS); double: 64 x 8 (512 threads, 104 KiB; a double 128 x 8
// tile does not fit in 160 KiB).  The float64 verification of a strain keeps
// 32 x 8 (VerifyTile): 64 x 8 ran it slower.
template <typename T>
struct Tile;
template <>
struct Tile<float> {
  static constexpr int DX = 128, DY = 8;
};
template <>
struct Tile<double> {
  static constexpr int DX = 64, DY = 8;
};
struct VerifyTile {
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
template <typename TC, int DX, int DY>
struct DivLds {
  TC st[6][DY + 1][DX + 1];
  TC ss[6][DY + 1][DX + 1];
  double red[7 * 16];
};

// One workgroup of the divergence walk: corner tile `tile` (x fastest, then
// y, then the z chunk), DX * DY threads, pointers already at the sample;
// writes its seven partial sums to out7.
template <int DX, int DY, typename TS, typename TC, typename TD, int OP>
__device__ __forceinline__ void div_body(DivLds<TC, DX, DY>& L, const TS* __restrict__ eps,
                                         const uint8_t* __restrict__ phase, const PhaseCoef<TC>* __restrict__ coef,
                                         TD* __restrict__ Dtau, TS* __restrict__ Dsig,
                                         const TS* __restrict__ Dsig_base, double* __restrict__ out7, const Dims& d,
                                         int zchunk, int tile) {
  constexpr int ER = (DX + 1) * (DY + 1), NT = DX * DY, ES = (ER + NT - 1) / NT;
  auto& st = L.st;
  auto& ss = L.ss;
  auto& red = L.red;
  const long long N = d.N;
  const int nx = d.nx, ny = d.ny, nz = d.nz;
  const int ntx = (nx + DX - 1) / DX, nty = (ny + DY - 1) / DY;
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
    for (int i = 0; i < 7; ++i) out7[i] = acc[i];
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
template <typename T, int DX, int DY>
struct UpdLds {
  T su[2][3][DY + 2][DX + 2];  // component-major: consecutive lanes hit consecutive banks
  T st[6][DY + 1][DX + 1];
  T ss[6][DY + 1][DX + 1];
  PhaseCoef<T> sc[256];
  double red[7 * 16];
};

// One workgroup of the fused update: corner tile `tile`, DX * DY threads,
// pointers already at the sample; writes its seven partial sums to out7.
template <int DX, int DY, typename T, int OP, bool AS, bool RF, bool WE>
__device__ __forceinline__ void update_div_body(UpdLds<T, DX, DY>& L, const T* __restrict__ U,
                                                const T* __restrict__ eps_in, T* __restrict__ eps_out,
                                                const uint8_t* __restrict__ phase,
                                                const PhaseCoef<T>* __restrict__ coef, int ncoef, const GreenConst<T>& g,
                                                const T* __restrict__ rfield, T* __restrict__ Dtau,
                                                const T* __restrict__ Dsig_base, double* __restrict__ out7,
                                                const Dims& d, int zchunk, int tile) {
  const long long N = d.N;
  constexpr int UR = (DX + 2) * (DY + 2), ER = (DX + 1) * (DY + 1), NT = DX * DY;
  constexpr int US = (UR + NT - 1) / NT, ES = (ER + NT - 1) / NT;  // per-thread slots
  auto& su = L.su;
  auto& st = L.st;
  auto& ss = L.ss;
  auto& sc = L.sc;
  auto& red = L.red;
  const int nx = d.nx, ny = d.ny, nz = d.nz;
  const int ntx = (nx + DX - 1) / DX, nty = (ny + DY - 1) / DY;
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
    for (int i = 0; i < 7; ++i) out7[i] = acc[i];
  }
}


// Tiling of the divergence walk: one corner tile and z chunk per workgroup,
// z cut into chunks of 8 to 64 planes so that a launch has at least about 2M
// threads (several generations of resident workgroups on 256 CUs).
struct DivGrid {
  int blocks, zchunk;
};
template <int DX, int DY>
inline DivGrid div_grid(const Dims& d) {
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



// Fixed-order sum of nblocks records of nv doubles (nv <= 8) by one workgroup
// of 256 threads: thread t adds records t, t + 256, ..., then the tree of
// block_sum; acc valid in thread 0 (the reduction every eta goes through).
__device__ __forceinline__ void reduce_body(const double* __restrict__ partials, int nblocks, int nv,
                                            double (&acc)[8], double* red) {
#pragma unroll
  for (int i = 0; i < 8; ++i) acc[i] = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x)
    for (int i = 0; i < nv && i < 8; ++i) acc[i] += partials[(long long)b * nv + i];
  block_sum<8>(acc, red);
}

// Corner tile of the divergence walk for a grid: Tile<T>, or 32 x 8 (256
// threads) for grids at most 128 wide (the tile of the persistent batched
// kernel; a wider tile would leave most of a small grid's row idle).
template <typename T>
struct SmallTile {
  static constexpr int DX = 32, DY = 8;
};
template <typename T, class F>
inline void with_tile(const Dims& d, F&& f) {
  if (d.nx <= 128)
    f(std::integral_constant<int, SmallTile<T>::DX>(), std::integral_constant<int, SmallTile<T>::DY>());
  else
    f(std::integral_constant<int, Tile<T>::DX>(), std::integral_constant<int, Tile<T>::DY>());
}

}  // namespace fe
