// Register-resident mixed-radix Stockham FFT with compile-time length for
// gfx950.
//
// A length-N sequence is processed by P = N/E threads; thread t holds the E
// elements at positions t + P*m (m = 0..E-1) in registers.  Stage s applies
// radix R_s butterflies (E/R_s per thread): butterfly j = t + i*P reads the
// elements j + r*N/R_s (register i + r*E/R_s), multiplies element r by
// exp(-+2 pi i r (j mod Ns)/(Ns R_s)) (Ns = product of the earlier radices) and
// applies the radix-R_s DFT (Stockham autosort, Govindaraju et al., SC 2008).
// Outputs go to positions (j/Ns) Ns R_s + (j mod Ns) + r Ns; between stages
// they pass through LDS (write, barrier, read back t + P*m, barrier).  After
// the last stage the outputs are already in natural order in the same
// registers (positions t + P*m), so loads and stores at both ends go straight
// between HBM and registers and no LDS round trip is needed there.
#pragma once

#include "fe_device.h"

namespace fe {

// ---------------------------------------------------------------------------
// radix-16 butterfly (4 x 4 with internal twiddles W16^(n1 k1))
// ---------------------------------------------------------------------------
template <typename T, bool INV>
__device__ __forceinline__ cpx<T> w16(cpx<T> a, int m) {
  const T c1 = T(0.92387953251128675612818318939679);  // cos(pi/8)
  const T s1 = T(0.38268343236508977172845998403040);  // sin(pi/8)
  const T h = T(0.70710678118654752440084436210485);
  // exp(-+ i pi m / 8)
  T c, s;
  switch (m) {
    case 1: c = c1; s = s1; break;
    case 2: c = h; s = h; break;
    case 3: c = s1; s = c1; break;
    case 4: return rot90<T, INV>(a);
    case 6: c = -h; s = h; break;
    case 9: c = -c1; s = -s1; break;
    default: return a;
  }
  const T sn = INV ? s : -s;  // w = c + i sn
  return mk(a.re * c - a.im * sn, a.re * sn + a.im * c);
}

template <typename T, bool INV>
struct Dft<T, 16, INV> {
  static __device__ __forceinline__ void run(cpx<T>* v) {
    cpx<T> a[4][4];
#pragma unroll
    for (int n1 = 0; n1 < 4; ++n1) {
      cpx<T> q[4] = {v[n1], v[n1 + 4], v[n1 + 8], v[n1 + 12]};
      Dft<T, 4, INV>::run(q);
#pragma unroll
      for (int k1 = 0; k1 < 4; ++k1) a[n1][k1] = w16<T, INV>(q[k1], n1 * k1);
    }
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      cpx<T> q[4] = {a[0][k1], a[1][k1], a[2][k1], a[3][k1]};
      Dft<T, 4, INV>::run(q);
#pragma unroll
      for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = q[k2];
    }
  }
};

// ---------------------------------------------------------------------------
// compile-time plan: radices chosen greedily (16, 8, 4, 2, then 3) among those
// dividing both the remaining length and E.
// ---------------------------------------------------------------------------
constexpr int pick_radix(int rem, int E) {
  return (rem % 16 == 0 && E % 16 == 0)   ? 16
         : (rem % 8 == 0 && E % 8 == 0)   ? 8
         : (rem % 4 == 0 && E % 4 == 0)   ? 4
         : (rem % 2 == 0 && E % 2 == 0)   ? 2
         : (rem % 3 == 0 && E % 3 == 0)   ? 3
                                          : 0;
}
constexpr int plan_radix(int N, int E, int s) {
  int rem = N;
  for (int i = 0; i < s; ++i) {
    const int r = pick_radix(rem, E);
    if (r == 0) return 0;
    rem /= r;
  }
  return rem == 1 ? 0 : pick_radix(rem, E);
}
constexpr int plan_ns(int N, int E, int s) {
  int p = 1;
  for (int i = 0; i < s; ++i) p *= plan_radix(N, E, i);
  return p;
}
constexpr int plan_stages(int N, int E) {
  int s = 0;
  while (plan_radix(N, E, s) != 0) ++s;
  return s;
}
constexpr bool plan_ok(int N, int E) { return N % E == 0 && plan_ns(N, E, plan_stages(N, E)) == N; }

// Elements per thread.
//  strided passes: up to 32 (2^a) or 24 (3*2^a); lengths up to 128 take 16
//  or 12, so that a 256-thread tile needs at most 32 KiB of LDS (four
//  workgroups per CU in the persistent batched kernel)
//  x passes: 8 (2^a) or 12 (3*2^a) with 3 components (float64: 4 or 6),
//  8 / 12 with 6
constexpr int e_strided(int N) {
  return N % 3 == 0 ? (N >= 192 ? 24 : (N >= 12 ? 12 : N)) : (N >= 256 ? 32 : (N >= 16 ? 16 : N));
}
constexpr int e_x3(int N) { return N % 3 == 0 ? (N >= 12 ? 12 : N) : (N >= 8 ? 8 : N); }
constexpr int e_x3_wide(int N) { return N % 3 == 0 ? (N >= 6 ? 6 : N) : (N >= 4 ? 4 : N); }
constexpr int e_x6(int N) { return N % 3 == 0 ? (N >= 12 ? 12 : N) : (N >= 8 ? 8 : N); }

// One Stockham stage over NC components held in registers.  `Lds` maps
// (component, position) to an LDS offset.  With SEQ the components take turns
// through one LDS buffer (less LDS, more barriers); otherwise all components
// exchange at once.
template <typename T, int N, int E, int S, int NC, bool INV, bool SEQ>
struct FftStage {
  static constexpr int R = plan_radix(N, E, S);
  static constexpr int NS = plan_ns(N, E, S);
  static constexpr int NST = plan_stages(N, E);
  static constexpr int B = E / R;
  static constexpr int P = N / E;
  static constexpr bool LAST = (S == NST - 1);

  template <class Lds>
  static __device__ __forceinline__ void butterflies(cpx<T> (&v)[NC][E], int c, int t, cpx<T>* lds, const Lds& at,
                                                     const cpx<T>* __restrict__ tw) {
#pragma unroll
    for (int i = 0; i < B; ++i) {
      const int j = t + i * P;
      const int k = j % NS;
      cpx<T> u[R];
#pragma unroll
      for (int r = 0; r < R; ++r) u[r] = v[c][i + r * B];
      if (NS > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          cpx<T> w = tw[r * k * (N / (NS * R))];
          if (INV) w.im = -w.im;
          u[r] = mul(u[r], w);
        }
      }
      Dft<T, R, INV>::run(u);
      if (LAST) {
#pragma unroll
        for (int r = 0; r < R; ++r) v[c][i + r * B] = u[r];
      } else {
        const int base = (j / NS) * NS * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) lds[at(c, base + r * NS)] = u[r];
      }
    }
  }

  template <class Lds>
  static __device__ __forceinline__ void run(cpx<T> (&v)[NC][E], int t, cpx<T>* lds, const Lds& at,
                                             const cpx<T>* __restrict__ tw) {
    if (LAST || !SEQ) {
#pragma unroll
      for (int c = 0; c < NC; ++c) butterflies(v, c, t, lds, at, tw);
      if (!LAST) {
        __syncthreads();
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
          for (int m = 0; m < E; ++m) v[c][m] = lds[at(c, t + m * P)];
        __syncthreads();
      }
    } else {
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        butterflies(v, c, t, lds, at, tw);
        __syncthreads();
#pragma unroll
        for (int m = 0; m < E; ++m) v[c][m] = lds[at(c, t + m * P)];
        __syncthreads();
      }
    }
  }
};

template <typename T, int N, int E, int S, int NC, bool INV, bool SEQ>
struct FftStages {
  template <class Lds>
  static __device__ __forceinline__ void run(cpx<T> (&v)[NC][E], int t, cpx<T>* lds, const Lds& at,
                                             const cpx<T>* __restrict__ tw) {
    if constexpr (S < plan_stages(N, E)) {
      FftStage<T, N, E, S, NC, INV, SEQ>::run(v, t, lds, at, tw);
      FftStages<T, N, E, S + 1, NC, INV, SEQ>::run(v, t, lds, at, tw);
    }
  }
};

// Full transform: v[c][m] holds input position t + P*m on entry and output
// position t + P*m on exit.  All threads of the block must call it (barriers);
// the LDS buffer is free again when it returns.
template <typename T, int N, int E, int NC, bool INV, bool SEQ = false, class Lds>
__device__ __forceinline__ void fft_regs(cpx<T> (&v)[NC][E], int t, cpx<T>* lds, const Lds& at,
                                         const cpx<T>* __restrict__ tw) {
  static_assert(plan_ok(N, E), "unsupported FFT length / elements per thread");
  FftStages<T, N, E, 0, NC, INV, SEQ>::run(v, t, lds, at, tw);
}

// Supported transform lengths (2^a and 3*2^a between 4 and 1024).
#define FE_FOR_EACH_LENGTH(X) \
  X(4) X(6) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(768) X(1024)

__host__ __device__ constexpr bool supported_length(int n) {
  return n == 4 || n == 6 || n == 8 || n == 12 || n == 16 || n == 24 || n == 32 || n == 48 || n == 64 ||
         n == 96 || n == 128 || n == 192 || n == 256 || n == 384 || n == 512 || n == 768 || n == 1024;
}
// z lengths: the above, and 1 (a one-plane cell, a 2D problem in plane strain)
__host__ __device__ constexpr bool supported_z_length(int n) { return n == 1 || supported_length(n); }

}  // namespace fe
