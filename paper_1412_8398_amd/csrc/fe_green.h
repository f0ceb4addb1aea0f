// Per-frequency Green operators and the spectral equilibrium norm
// (Willot, arXiv 1412.8398, §3-§4; equation numbers are the paper's).
#pragma once

#include "fe_kernels.h"

namespace fe {

// Voigt index of entry (i, j) of a symmetric tensor: (1,2)->3, (0,2)->4, (0,1)->5.
__host__ __device__ __forceinline__ int voigt_of(int i, int j) {
  if (i == j) return i;
  const int s = i + j;
  return s == 3 ? 3 : (s == 2 ? 4 : 5);
}

// Solve A x = b for the Hermitian 3x3 matrix of eq. (19),
//   A = lam0 conj(k) k^T + mu0 k conj(k)^T + mu0 |k|^2 I,
// by the Woodbury identity over its rank-2 part:
//   A^-1 b = (b - conj(k) y1 - k y2) / (mu0 |k|^2),
//   M y = [lam0 k^T b, mu0 k^H b],  M = [[(lam0+mu0)|k|^2, lam0 k.k], [mu0 conj(k.k), 2 mu0 |k|^2]].
template <typename T>
__device__ __forceinline__ void woodbury_solve(const cpx<T> (&k)[3], const cpx<T> (&b)[3], T lam0, T mu0,
                                               cpx<T> (&x)[3]) {
  const T n2 = norm2(k[0]) + norm2(k[1]) + norm2(k[2]);
  const cpx<T> s = add(add(mul(k[0], k[0]), mul(k[1], k[1])), mul(k[2], k[2]));
  const cpx<T> p = add(add(mul(k[0], b[0]), mul(k[1], b[1])), mul(k[2], b[2]));
  const cpx<T> r = add(add(mul(conj(k[0]), b[0]), mul(conj(k[1]), b[1])), mul(conj(k[2]), b[2]));
  const T det = T(2) * mu0 * (lam0 + mu0) * n2 * n2 - lam0 * mu0 * norm2(s);
  const T idet = T(1) / det;
  const cpx<T> y1 = scale(sub(scale(p, T(2) * mu0 * n2 * lam0), scale(mul(s, r), lam0 * mu0)), idet);
  const cpx<T> y2 = scale(sub(scale(r, (lam0 + mu0) * n2 * mu0), scale(mul(conj(s), p), mu0 * lam0)), idet);
  const T iD = T(1) / (mu0 * n2);
#pragma unroll
  for (int a = 0; a < 3; ++a) x[a] = scale(sub(sub(b[a], mul(conj(k[a]), y1)), mul(k[a], y2)), iD);
}

// 1/x: the hardware reciprocal (1 ulp) in float, a division in double.
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }

// k(q) from the per-axis tables.
//   MS : k = i q                        (eqs. (7)-(8))
//   C  : k = i sin q                    (centered differences, §4.2)
//   WP : k = exp(i q) - 1               (eq. (21))
//   ROT: k = 2 i exp(i (q1+q2+q3)/2) t, t_a = sin(q_a/2) prod_{b!=a} cos(q_b/2)  (eq. (36))
template <typename T, int OP>
__device__ __forceinline__ void wave_k(const WaveTables<T>& wt, int mx, int my, int mz, cpx<T> (&k)[3]) {
  const T ax = wt.x[2 * mx], bx = wt.x[2 * mx + 1];
  const T ay = wt.y[2 * my], by = wt.y[2 * my + 1];
  const T az = wt.z[2 * mz], bz = wt.z[2 * mz + 1];
  if (OP == OP_WP) {
    k[0] = mk(ax, bx);
    k[1] = mk(ay, by);
    k[2] = mk(az, bz);
  } else if (OP == OP_MS || OP == OP_C || OP == OP_MSS) {  // i q or i sin q
    k[0] = mk(T(0), ax);
    k[1] = mk(T(0), ay);
    k[2] = mk(T(0), az);
  } else {
    const T t0 = ax * by * bz, t1 = ay * bx * bz, t2 = az * bx * by;
    const cpx<T> ph = mul(mul(mk(bx, ax), mk(by, ay)), mk(bz, az));
    const cpx<T> f = mk(-T(2) * ph.im, T(2) * ph.re);
    k[0] = scale(f, t0);
    k[1] = scale(f, t1);
    k[2] = scale(f, t2);
  }
}

// Displacement form: from D(q) = FFT of the discrete divergence of tau, return
// u(q)/N with eps = eps_bar + sym grad_h u.
// ROT: D = conj(k)-divergence (symbol conj k^R), A = 4(lam0+mu0) t t^T + 4 mu0 |t|^2 I,
//      u = -A^-1 D = -(D - cr t (t.D)/|t|^2) / (4 mu0 |t|^2); u = 0 where t = 0 (q = 0 and
//      where two q_i equal pi, eq. (41)).
// WP:  D is the backward-difference divergence, symbol -conj(k^W): u = A^-1 D.
template <typename T, int OP>
__device__ __forceinline__ void green_disp(cpx<T> (&b)[3], const WaveTables<T>& wt, int mx, int my, int mz,
                                           const GreenConst<T>& g) {
  if (OP == OP_ROT) {
    const T ax = wt.x[2 * mx], bx = wt.x[2 * mx + 1];
    const T ay = wt.y[2 * my], by = wt.y[2 * my + 1];
    const T az = wt.z[2 * mz], bz = wt.z[2 * mz + 1];
    const T t[3] = {ax * by * bz, ay * bx * bz, az * bx * by};
    const T tt = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
    if (tt > T(0)) {
      const cpx<T> tb = add(add(scale(b[0], t[0]), scale(b[1], t[1])), scale(b[2], t[2]));
      const T itt = recip(tt);
      const T f = -g.inv_n / (T(4) * g.mu0) * itt;
      const T h = g.cr * itt;
#pragma unroll
      for (int a = 0; a < 3; ++a) b[a] = scale(sub(b[a], scale(tb, h * t[a])), f);
    } else {
#pragma unroll
      for (int a = 0; a < 3; ++a) b[a] = mk(T(0), T(0));
    }
  } else {
    if (mx == 0 && my == 0 && mz == 0) {
#pragma unroll
      for (int a = 0; a < 3; ++a) b[a] = mk(T(0), T(0));
    } else {
      cpx<T> k[3], u[3];
      wave_k<T, OP_WP>(wt, mx, my, mz, k);
      woodbury_solve(k, b, g.lam0, g.mu0, u);
#pragma unroll
      for (int a = 0; a < 3; ++a) b[a] = scale(u[a], g.inv_n);
    }
  }
}

// eps/N = -sym(k (x) u)/N with u = -A^-1 conj(k).tau (eq. (19)), for |k| > 0.
template <typename T>
__device__ __forceinline__ void green_sym_solve(const cpx<T> (&k)[3], const cpx<T> (&tv)[6], const GreenConst<T>& g,
                                                cpx<T> (&out)[6]) {
  cpx<T> b[3], u[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    cpx<T> acc = mk(T(0), T(0));
#pragma unroll
    for (int i = 0; i < 3; ++i) acc = add(acc, mul(conj(k[i]), tv[voigt_of(i, j)]));
    b[j] = acc;
  }
  woodbury_solve(k, b, g.lam0, g.mu0, u);
  const T f = -g.inv_n;
  out[0] = scale(mul(k[0], u[0]), f);
  out[1] = scale(mul(k[1], u[1]), f);
  out[2] = scale(mul(k[2], u[2]), f);
  out[3] = scale(add(mul(k[1], u[2]), mul(k[2], u[1])), T(0.5) * f);
  out[4] = scale(add(mul(k[0], u[2]), mul(k[2], u[0])), T(0.5) * f);
  out[5] = scale(add(mul(k[0], u[1]), mul(k[1], u[0])), T(0.5) * f);
}

// Nyquist flag of the MS wave tables at (mx, my, mz): some q_i = pi (even L_i)
template <typename T>
__device__ __forceinline__ bool nyquist_mode(const WaveTables<T>& wt, int mx, int my, int mz) {
  return (wt.x[2 * mx + 1] != T(0)) || (wt.y[2 * my + 1] != T(0)) || (wt.z[2 * mz + 1] != T(0));
}

// Six-component form (any operator): tau(q) -> eps(q)/N.
//   q = 0: eps_bar (eq. (6));  MS with some q_i = pi: -(C0)^-1 tau (eq. (14));
//   ordinary: b_j = conj(k_i) tau_ij, u = -A^-1 b, eps = sym(k (x) u) (eq. (19));
//   ROT with two q_i = pi: |k| = 0, eps = 0 (eq. (41));
//   C with every q_i in {0, pi}: |k| = 0, eps = 0 (eq. (29));
//   MSS with some q_i = pi: the mean of the ordinary formula at k = i q and at
//   k' = i q', q' = -q with the Nyquist components kept at +pi (the grid
//   partner of q; eq. (15)).
template <typename T, int OP>
__device__ __forceinline__ void green_six(cpx<T> (&tv)[6], const WaveTables<T>& wt, int mx, int my, int mz,
                                          const GreenConst<T>& g) {
  if (mx == 0 && my == 0 && mz == 0) {
#pragma unroll
    for (int c = 0; c < 6; ++c) tv[c] = mk(g.macro[c], T(0));
    return;
  }
  if (OP == OP_MSS && nyquist_mode(wt, mx, my, mz)) {
    const T qx = wt.x[2 * mx], qy = wt.y[2 * my], qz = wt.z[2 * mz];
    const cpx<T> k[3] = {mk(T(0), qx), mk(T(0), qy), mk(T(0), qz)};
    const cpx<T> kp[3] = {mk(T(0), wt.x[2 * mx + 1] != T(0) ? qx : -qx),
                          mk(T(0), wt.y[2 * my + 1] != T(0) ? qy : -qy),
                          mk(T(0), wt.z[2 * mz + 1] != T(0) ? qz : -qz)};
    cpx<T> e1[6], e2[6];
    green_sym_solve(k, tv, g, e1);
    green_sym_solve(kp, tv, g, e2);
#pragma unroll
    for (int c = 0; c < 6; ++c) tv[c] = scale(add(e1[c], e2[c]), T(0.5));
    return;
  }
  if (OP == OP_MS) {
    const bool nyq = nyquist_mode(wt, mx, my, mz);
    if (nyq) {
      const cpx<T> tr = add(add(tv[0], tv[1]), tv[2]);
#pragma unroll
      for (int c = 0; c < 6; ++c) tv[c] = scale(tv[c], -g.s1 * g.inv_n);
#pragma unroll
      for (int c = 0; c < 3; ++c) tv[c] = add(tv[c], scale(tr, g.s2 * g.inv_n));
      return;
    }
  }
  cpx<T> k[3];
  wave_k<T, OP>(wt, mx, my, mz, k);
  const T n2 = norm2(k[0]) + norm2(k[1]) + norm2(k[2]);
  if (!(n2 > T(0))) {
#pragma unroll
    for (int c = 0; c < 6; ++c) tv[c] = mk(T(0), T(0));
    return;
  }
  cpx<T> e[6];
  green_sym_solve(k, tv, g, e);
#pragma unroll
  for (int c = 0; c < 6; ++c) tv[c] = e[c];
}

// |conj(k).sigma(q)|^2 summed over the stored q and, for 0 < mz < nz/2, its
// mirror -q (coefficient conj sigma(q), wave vector read at the mirror
// indices) -- eq. (43) over the full spectrum from a half spectrum.
// The two divergence vectors behind eta_six: conj(k(q)).sigma(q) into a[0..2]
// and, where the half spectrum stands for the mirror -q too (0 < mz < nz/2),
// conj(k(-q)).conj(sigma(q)) into b[0..2] (else b = 0).  Returns whether b
// is used.
template <typename T, int OP>
__device__ __forceinline__ bool div_six(const cpx<T> (&sv)[6], const WaveTables<T>& wt, int mx, int my, int mz,
                                        const Dims& d, cpx<T> (&a)[3], cpx<T> (&b)[3]) {
  cpx<T> k[3];
  wave_k<T, OP>(wt, mx, my, mz, k);
  const bool off = OP == OP_MSS && nyquist_mode(wt, mx, my, mz);  // as eta_six
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    a[j] = mk(T(0), T(0));
    if (!off) {
#pragma unroll
      for (int i = 0; i < 3; ++i) a[j] = add(a[j], mul(conj(k[i]), sv[voigt_of(i, j)]));
    }
    b[j] = mk(T(0), T(0));
  }
  if (off || !(mz > 0 && 2 * mz < d.nz)) return false;
  const int qx = mx == 0 ? 0 : d.nx - mx, qy = my == 0 ? 0 : d.ny - my, qz = d.nz - mz;
  wave_k<T, OP>(wt, qx, qy, qz, k);
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int i = 0; i < 3; ++i) b[j] = add(b[j], mul(conj(k[i]), conj(sv[voigt_of(i, j)])));
  return true;
}

template <typename T, int OP>
__device__ __forceinline__ double eta_six(const cpx<T> (&sv)[6], const WaveTables<T>& wt, int mx, int my, int mz,
                                          const Dims& d) {
  // MSS imposes equilibrium off the Nyquist modes only (a mode and its
  // mirror are Nyquist together): eq. (43) sums over the others
  if (OP == OP_MSS && nyquist_mode(wt, mx, my, mz)) return 0.0;
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
  if (mz > 0 && 2 * mz < d.nz) {
    const int qx = mx == 0 ? 0 : d.nx - mx, qy = my == 0 ? 0 : d.ny - my, qz = d.nz - mz;
    wave_k<T, OP>(wt, qx, qy, qz, k);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      cpx<T> a = mk(T(0), T(0));
#pragma unroll
      for (int i = 0; i < 3; ++i) a = add(a, mul(conj(k[i]), conj(sv[voigt_of(i, j)])));
      s += double(a.re) * double(a.re) + double(a.im) * double(a.im);
    }
  }
  return s;
}

}  // namespace fe
