// Device building blocks for the gfx950 solver: complex arithmetic, small DFT
// butterflies and deterministic float64 block reductions.
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

// Workgroups are dispatched round-robin over the 8 XCDs (workgroup b runs on
// XCD b mod 8), each with its own L2.  This renumbering hands every XCD a
// contiguous range of logical blocks, so tiles that share halo lines (x and y
// neighbours) are resident on the same L2 at about the same time.  It is a
// bijection of [0, nb).
__device__ __forceinline__ int xcd_block(int b, int nb) {
  const int q = nb >> 3, r = nb & 7, k = b & 7;
  return k * q + (k < r ? k : r) + (b >> 3);
}

}  // namespace fe
