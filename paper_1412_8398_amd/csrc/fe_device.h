// Device building blocks for the gfx950 solver: complex arithmetic, small DFT
// butterflies, one mixed-radix Stockham stage over a tile held in LDS, and
// deterministic float64 block reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fe {

template <typename T>
struct alignas(2 * sizeof(T)) cpx {
  T re, im;
};

template <typename T>
__device__ __forceinline__ cpx<T> mk(T r, T i) {
  cpx<T> c;
  c.re = r;
  c.im = i;
  return c;
}
template <typename T>
__device__ __forceinline__ cpx<T> add(cpx<T> a, cpx<T> b) { return mk(a.re + b.re, a.im + b.im); }
template <typename T>
__device__ __forceinline__ cpx<T> sub(cpx<T> a, cpx<T> b) { return mk(a.re - b.re, a.im - b.im); }
template <typename T>
__device__ __forceinline__ cpx<T> mul(cpx<T> a, cpx<T> b) {
  return mk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <typename T>
__device__ __forceinline__ cpx<T> conj(cpx<T> a) { return mk(a.re, -a.im); }
template <typename T>
__device__ __forceinline__ cpx<T> scale(cpx<T> a, T s) { return mk(a.re * s, a.im * s); }
// multiply by -i (forward) or +i (inverse)
template <typename T, bool INV>
__device__ __forceinline__ cpx<T> rot90(cpx<T> a) {
  return INV ? mk(-a.im, a.re) : mk(a.im, -a.re);
}
template <typename T>
__device__ __forceinline__ T norm2(cpx<T> a) { return a.re * a.re + a.im * a.im; }

// ---------------------------------------------------------------------------
// DFT butterflies: y_k = sum_r v_r exp(-+ 2 pi i r k / R), sign + for INV.
// ---------------------------------------------------------------------------
template <typename T, int R, bool INV>
struct Dft;

template <typename T, bool INV>
struct Dft<T, 2, INV> {
  static __device__ __forceinline__ void run(cpx<T>* v) {
    cpx<T> a = v[0], b = v[1];
    v[0] = add(a, b);
    v[1] = sub(a, b);
  }
};

template <typename T, bool INV>
struct Dft<T, 3, INV> {
  static __device__ __forceinline__ void run(cpx<T>* v) {
    const T s3 = T(0.86602540378443864676372317075294);  // sin(2 pi / 3)
    cpx<T> t1 = add(v[1], v[2]);
    cpx<T> t2 = sub(v[0], scale(t1, T(0.5)));
    cpx<T> t3 = scale(sub(v[1], v[2]), s3);
    cpx<T> r = rot90<T, INV>(t3);  // -+ i (sqrt3/2)(v1 - v2)
    v[0] = add(v[0], t1);
    v[1] = add(t2, r);
    v[2] = sub(t2, r);
  }
};

template <typename T, bool INV>
struct Dft<T, 4, INV> {
  static __device__ __forceinline__ void run(cpx<T>* v) {
    cpx<T> a0 = add(v[0], v[2]), a1 = sub(v[0], v[2]);
    cpx<T> b0 = add(v[1], v[3]), b1 = rot90<T, INV>(sub(v[1], v[3]));
    v[0] = add(a0, b0);
    v[2] = sub(a0, b0);
    v[1] = add(a1, b1);
    v[3] = sub(a1, b1);
  }
};

template <typename T, bool INV>
struct Dft<T, 8, INV> {
  static __device__ __forceinline__ void run(cpx<T>* v) {
    const T h = T(0.70710678118654752440084436210485);  // sqrt(1/2)
    cpx<T> e[4] = {v[0], v[2], v[4], v[6]};
    cpx<T> o[4] = {v[1], v[3], v[5], v[7]};
    Dft<T, 4, INV>::run(e);
    Dft<T, 4, INV>::run(o);
    // twiddles w^k, w = exp(-+ 2 pi i / 8)
    cpx<T> o1 = INV ? mk(h * (o[1].re - o[1].im), h * (o[1].re + o[1].im))
                    : mk(h * (o[1].re + o[1].im), h * (o[1].im - o[1].re));
    cpx<T> o2 = rot90<T, INV>(o[2]);
    cpx<T> o3 = INV ? mk(-h * (o[3].re + o[3].im), h * (o[3].re - o[3].im))
                    : mk(h * (o[3].im - o[3].re), -h * (o[3].re + o[3].im));
    v[0] = add(e[0], o[0]);
    v[4] = sub(e[0], o[0]);
    v[1] = add(e[1], o1);
    v[5] = sub(e[1], o1);
    v[2] = add(e[2], o2);
    v[6] = sub(e[2], o2);
    v[3] = add(e[3], o3);
    v[7] = sub(e[3], o3);
  }
};

// ---------------------------------------------------------------------------
// One Stockham autosort stage (Govindaraju et al., SC 2008 formulation) over
// `ncol` independent length-n sequences in LDS, element (e, col) at
// lds[e*es + col*cs].  With Ns the product of the radices already applied,
// butterfly j reads elements j + r n/R, multiplies element r by
// exp(-+2 pi i r (j mod Ns) / (Ns R)), applies a radix-R DFT and writes
// element r to (j/Ns) Ns R + (j mod Ns) + r Ns.  Reads complete (barrier)
// before writes, so the stage runs in place.  Callers barrier before the
// first stage; every stage ends with a barrier.
// `tw` holds exp(-2 pi i k / n), k < n (host float64, rounded to T).
// ---------------------------------------------------------------------------
template <typename T, int R, int MAXB, bool INV>
__device__ __forceinline__ void stockham_stage(cpx<T>* lds, int n, int ncol, int es, int cs, int Ns,
                                               const cpx<T>* __restrict__ tw, int tid, int nthr) {
  const int nq = n / R;
  const int nbf = ncol * nq;
  const int tstep = n / (Ns * R);
  cpx<T> v[MAXB][R];
  int dst[MAXB];
#pragma unroll
  for (int i = 0; i < MAXB; ++i) {
    const int b = tid + i * nthr;
    dst[i] = -1;
    if (b < nbf) {
      const int col = b % ncol;
      const int j = b / ncol;
      const int k = j % Ns;
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = lds[(j + r * nq) * es + col * cs];
      const int step = k * tstep;
#pragma unroll
      for (int r = 1; r < R; ++r) {
        cpx<T> w = tw[r * step];
        if (INV) w.im = -w.im;
        v[i][r] = mul(v[i][r], w);
      }
      Dft<T, R, INV>::run(v[i]);
      dst[i] = ((j / Ns) * Ns * R + k) * es + col * cs;
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < MAXB; ++i) {
    if (dst[i] >= 0) {
#pragma unroll
      for (int r = 0; r < R; ++r) lds[dst[i] + r * Ns * es] = v[i][r];
    }
  }
  __syncthreads();
}

// Radix plan of a length: up to 8 stages, 4 bits each, radices in {2,3,4,8}.
__host__ __device__ inline int radix_at(uint32_t plan, int s) { return (plan >> (4 * s)) & 0xF; }

// Full in-place FFT of a tile in LDS.  NTHR threads; CAP = max ncol*n.
template <typename T, bool INV, int NTHR, int CAP>
__device__ __forceinline__ void fft_tile(cpx<T>* lds, int n, int ncol, int es, int cs,
                                         const cpx<T>* __restrict__ tw, uint32_t plan) {
  const int tid = threadIdx.x;
  int Ns = 1;
#pragma unroll 1
  for (int s = 0; s < 8; ++s) {
    const int R = radix_at(plan, s);
    if (R == 0) break;
    switch (R) {
      case 8: stockham_stage<T, 8, (CAP + 8 * NTHR - 1) / (8 * NTHR), INV>(lds, n, ncol, es, cs, Ns, tw, tid, NTHR); break;
      case 4: stockham_stage<T, 4, (CAP + 4 * NTHR - 1) / (4 * NTHR), INV>(lds, n, ncol, es, cs, Ns, tw, tid, NTHR); break;
      case 3: stockham_stage<T, 3, (CAP + 3 * NTHR - 1) / (3 * NTHR), INV>(lds, n, ncol, es, cs, Ns, tw, tid, NTHR); break;
      default: stockham_stage<T, 2, (CAP + 2 * NTHR - 1) / (2 * NTHR), INV>(lds, n, ncol, es, cs, Ns, tw, tid, NTHR); break;
    }
    Ns *= R;
  }
}

// ---------------------------------------------------------------------------
// Deterministic float64 reductions: wavefront shuffle tree, then a fixed
// order over the block's waves through LDS.  Result valid in thread 0.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* scratch /* >= NV*16 */) {
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) scratch[i * 16 + wid] = v[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      double s = 0.0;
      for (int w = 0; w < nw; ++w) s += scratch[i * 16 + w];
      v[i] = s;
    }
  }
}

}  // namespace fe
