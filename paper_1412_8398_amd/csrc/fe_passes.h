// FFT pass kernels (compile-time lengths) and their launchers.
//
// Spectrum layout: half spectra along z, [comp][mz][y][x] complex, mz in
// [0, nz/2].  Real planes: [comp][z][y][x].
#pragma once

#include <type_traits>

#include "fe_fft.h"
#include "fe_green.h"

namespace fe {

template <typename T>
constexpr int lds_budget() {  // complex elements per workgroup tile
  return (64 * 1024) / (int)sizeof(cpx<T>);
}
constexpr int imin(int a, int b) { return a < b ? a : b; }
constexpr int imax(int a, int b) { return a > b ? a : b; }

// Strided passes: TX adjacent x-columns per workgroup, P = N/E threads per
// column, E elements per thread; 256 threads unless the LDS tile caps TX.
template <typename T, int N, bool YPASS = false>
struct StridedCfg {
  static constexpr int E = e_strided(N);
  static constexpr int P = N / E;
  // long y columns: 512 threads and up to 128 KiB of LDS keep 16 columns
  // (128-byte rows in float) per workgroup (measured: faster for y at 1024,
  // slower for the z passes, whose 64-byte halves pair up in L2 anyway)
  static constexpr bool BIG = YPASS && N >= 768;
  static constexpr int TX = imax(1, imin((BIG ? 512 : 256) / P, (BIG ? 2 : 1) * lds_budget<T>() / N));
  static constexpr int NT = TX * P;
  // LDS rows of TX complex values; with TX <= 16 (lengths >= 384) one empty
  // row follows every 16, so that the two rows a 16-lane quarter of a wave
  // touches in an exchange fall on different halves of the 32 banks (rows
  // 16 or 32 positions apart would otherwise share them)
  static constexpr int RPAD = TX <= 16 ? 16 : 0;
  static constexpr int ROWS = N + (RPAD ? N / RPAD : 0);
  static __device__ __forceinline__ int row(int pos) { return RPAD ? pos + pos / RPAD : pos; }
};

// x passes: LPB lines per workgroup, P = N/E threads per line.
template <typename T, int N, int NC>
struct LineCfg {
  // float64 lines of three components hold half the elements per thread: a
  // workgroup of 4 lines at 8 elements would take 96 KiB of LDS at 512 (one
  // workgroup, one wave per SIMD)
  static constexpr int E = NC == 3 ? (sizeof(T) == 8 ? e_x3_wide(N) : e_x3(N)) : e_x6(N);
  static constexpr int P = N / E;
  static constexpr int LPB = imax(1, 256 / P);
  static constexpr int NT = LPB * P;
  // LDS position of element pos of a line: lines of 128 and more permute
  // each aligned block of 32 by an XOR with bits 3-7 of pos (no padding; the
  // strided writes of every exchange stage then spread over all 32 banks
  // within each 16-lane quarter wave), shorter lines pad one element per 16
  static constexpr bool SWZ = N >= 128;
  static constexpr int LINE = SWZ ? N : N + N / 16;
  static __device__ __forceinline__ int pos(int p) { return SWZ ? p ^ ((p >> 3) & 31) : p + (p >> 4); }
};

template <typename T>
struct alignas(4 * sizeof(T)) cpx2 {
  cpx<T> a, b;
};

// ---------------------------------------------------------------------------
// y: complex transform of the half spectrum along y, in place
// ---------------------------------------------------------------------------
// One workgroup (tile lb) of the y pass on one sample's spectra S.
template <typename T, int N, bool INV>
__device__ __forceinline__ void ypass_body(cpx<T>* __restrict__ S, const Dims& d, const cpx<T>* __restrict__ tw,
                                           cpx<T>* lds, int lb) {
  using C = StridedCfg<T, N, true>;
  const int col = threadIdx.x % C::TX, t = threadIdx.x / C::TX;
  const int ntx = (d.nx + C::TX - 1) / C::TX;
  const int xt = lb % ntx;
  const int rest = lb / ntx;
  const int mz = rest % d.H;
  const int c = rest / d.H;
  const int x = xt * C::TX + col;
  const bool ok = x < d.nx;
  cpx<T>* base = S + (long long)c * spec_size(d) + zidx(d, mz, 0, ok ? x : 0);
  const long long ys = (long long)d.nx << d.zs;  // consecutive y rows of one plane
  cpx<T> v[1][C::E];
#pragma unroll
  for (int m = 0; m < C::E; ++m) v[0][m] = ok ? base[(long long)(t + m * C::P) * ys] : mk(T(0), T(0));
  fft_regs<T, N, C::E, 1, INV>(v, t, lds, [col](int, int pos) { return C::row(pos) * C::TX + col; }, tw);
  if (ok) {
#pragma unroll
    for (int m = 0; m < C::E; ++m) base[(long long)(t + m * C::P) * ys] = v[0][m];
  }
}

template <typename T, int N, bool INV>
__global__ __launch_bounds__((StridedCfg<T, N, true>::NT)) void k_ypass(cpx<T>* __restrict__ S, Dims d,
                                                                      const cpx<T>* __restrict__ tw, Batch bt) {
  using C = StridedCfg<T, N, true>;
  if (bt.active) S += (long long)bt.active[blockIdx.y] * (gridDim.x / (((d.nx + C::TX - 1) / C::TX) * d.H)) * spec_size(d);
  __shared__ cpx<T> lds[C::ROWS * C::TX];
  // x-neighbour tiles share 128-byte lines: same L2
  ypass_body<T, N, INV>(S, d, tw, lds, xcd_block(blockIdx.x, gridDim.x));
}

// ---------------------------------------------------------------------------
// z: real-to-complex.  Two adjacent real x-columns are one complex column
// z = a + i b; after the transform A(m) = (Z(m) + conj Z(-m))/2 and
// B(m) = (Z(m) - conj Z(-m))/(2i) for m in [0, nz/2].
// ---------------------------------------------------------------------------
// One workgroup (tile lb) of the real-to-complex z pass on one sample (R its
// real planes, S its half spectra).
template <typename T, int N>
__device__ __forceinline__ void zr2c_body(const T* __restrict__ R, cpx<T>* __restrict__ S, const Dims& d,
                                          const cpx<T>* __restrict__ tw, cpx<T>* lds, int lb) {
  using C = StridedCfg<T, N>;
  const int col = threadIdx.x % C::TX, t = threadIdx.x / C::TX;
  const int npair = d.nx / 2;
  const int ntx = (npair + C::TX - 1) / C::TX;
  const int xt = lb % ntx;
  const int rest = lb / ntx;
  const int y = rest % d.ny;
  const int c = rest / d.ny;
  const int pp = xt * C::TX + col;
  const bool ok = pp < npair;
  const T* src = R + (long long)c * d.N + 2 * (ok ? pp : 0);
  cpx<T> v[1][C::E];
#pragma unroll
  for (int m = 0; m < C::E; ++m)
    v[0][m] = ok ? *reinterpret_cast<const cpx<T>*>(src + zrow(d, t + m * C::P, y) * d.nx) : mk(T(0), T(0));
  fft_regs<T, N, C::E, 1, false>(v, t, lds, [col](int, int pos) { return C::row(pos) * C::TX + col; }, tw);
#pragma unroll
  for (int m = 0; m < C::E; ++m) lds[C::row(t + m * C::P) * C::TX + col] = v[0][m];
  __syncthreads();
  cpx<T>* dst = S + (long long)c * spec_size(d) + 2 * (ok ? pp : 0);
  constexpr int H = N / 2 + 1, NS = (H + C::P - 1) / C::P;
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    const int mz = t + i * C::P;
    if (mz >= H) break;
    const cpx<T> Z = lds[C::row(mz) * C::TX + col];
    const cpx<T> Zm = conj(lds[C::row((N - mz) % N) * C::TX + col]);
    const cpx<T> Dd = sub(Z, Zm);
    cpx2<T> o;
    o.a = scale(add(Z, Zm), T(0.5));
    o.b = mk(T(0.5) * Dd.im, T(-0.5) * Dd.re);
    if (ok) *reinterpret_cast<cpx2<T>*>(dst + zrow(d, mz, y) * d.nx) = o;
  }
}


template <typename T, int N>
__global__ __launch_bounds__((StridedCfg<T, N>::NT)) void k_zr2c(const T* __restrict__ R, cpx<T>* __restrict__ S,
                                                               Dims d, const cpx<T>* __restrict__ tw, Batch bt) {
  using C = StridedCfg<T, N>;
  if (bt.active) {
    const long long nc = gridDim.x / (((d.nx / 2 + C::TX - 1) / C::TX) * d.ny);
    const long long smp = bt.active[blockIdx.y];
    R += smp * nc * d.N;
    S += smp * nc * spec_size(d);
  }
  __shared__ cpx<T> lds[C::ROWS * C::TX];
  // x-neighbour tiles share 128-byte lines: same L2
  zr2c_body<T, N>(R, S, d, tw, lds, xcd_block(blockIdx.x, gridDim.x));
}

// z: complex-to-real (unnormalised inverse): Z(m) = A(m) + i B(m),
// Z(nz-m) = conj A(m) + i conj B(m); the inverse transform of Z is a + i b.
template <typename T, int N>
__device__ __forceinline__ void zc2r_body(const cpx<T>* __restrict__ S, T* __restrict__ R, const Dims& d,
                                          const cpx<T>* __restrict__ tw, cpx<T>* lds, int lb) {
  using C = StridedCfg<T, N>;
  const int col = threadIdx.x % C::TX, t = threadIdx.x / C::TX;
  const int npair = d.nx / 2;
  const int ntx = (npair + C::TX - 1) / C::TX;
  const int xt = lb % ntx;
  const int rest = lb / ntx;
  const int y = rest % d.ny;
  const int c = rest / d.ny;
  const int pp = xt * C::TX + col;
  const bool ok = pp < npair;
  const cpx<T>* src = S + (long long)c * spec_size(d) + 2 * (ok ? pp : 0);
  // all loads of this thread in flight before the first LDS store (H = N/2 + 1
  // half-spectrum planes, ceil(H/P) per thread)
  constexpr int H = N / 2 + 1, NL = (H + C::P - 1) / C::P;
  cpx2<T> ab[NL];
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    const int mz = t + i * C::P;
    if (ok && mz < H) {
      ab[i] = *reinterpret_cast<const cpx2<T>*>(src + zrow(d, mz, y) * d.nx);
    } else {
      ab[i].a = mk(T(0), T(0));
      ab[i].b = mk(T(0), T(0));
    }
  }
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    const int mz = t + i * C::P;
    if (mz < H) {
      const cpx<T> A = ab[i].a, B = ab[i].b;
      lds[C::row(mz) * C::TX + col] = mk(A.re - B.im, A.im + B.re);
      if (mz > 0 && 2 * mz < N) lds[C::row(N - mz) * C::TX + col] = mk(A.re + B.im, B.re - A.im);
    }
  }
  __syncthreads();
  cpx<T> v[1][C::E];
#pragma unroll
  for (int m = 0; m < C::E; ++m) v[0][m] = lds[C::row(t + m * C::P) * C::TX + col];
  __syncthreads();
  fft_regs<T, N, C::E, 1, true>(v, t, lds, [col](int, int pos) { return C::row(pos) * C::TX + col; }, tw);
  if (ok) {
    T* dst = R + (long long)c * d.N + 2 * pp;
#pragma unroll
    for (int m = 0; m < C::E; ++m) *reinterpret_cast<cpx<T>*>(dst + zrow(d, t + m * C::P, y) * d.nx) = v[0][m];
  }
}


template <typename T, int N>
__global__ __launch_bounds__((StridedCfg<T, N>::NT)) void k_zc2r(const cpx<T>* __restrict__ S, T* __restrict__ R,
                                                               Dims d, const cpx<T>* __restrict__ tw, Batch bt) {
  using C = StridedCfg<T, N>;
  if (bt.active) {
    const long long nc = gridDim.x / (((d.nx / 2 + C::TX - 1) / C::TX) * d.ny);
    const long long smp = bt.active[blockIdx.y];
    R += smp * nc * d.N;
    S += smp * nc * spec_size(d);
  }
  __shared__ cpx<T> lds[C::ROWS * C::TX];
  // x-neighbour tiles share 128-byte lines: same L2
  zc2r_body<T, N>(S, R, d, tw, lds, xcd_block(blockIdx.x, gridDim.x));
}

// ---------------------------------------------------------------------------
// x: forward transform of each contiguous x-line, Green operator per
// frequency in registers, inverse transform.
// ---------------------------------------------------------------------------

// x-line `line` of the z-blocked half spectrum (Hp ny lines per component) ->
// its plane mz and row y; false for the padding planes mz >= H and beyond the
// last line (then mz = y = 0).
__device__ __forceinline__ bool xline_of(const Dims& d, int line, int& mz, int& my) {
  mz = 0;
  my = 0;
  if (line >= d.Hp * d.ny) return false;
  const int r = line >> d.zs;
  const int z = ((r / d.ny) << d.zs) + (line & ((1 << d.zs) - 1));
  if (z >= d.H) return false;
  mz = z;
  my = r % d.ny;
  return true;
}
// One workgroup (line block bx) of the x pass with the Green operator of the
// displacement form on one sample's spectra S; lds holds 3 LPB LINE values,
// or LPB LINE with SEQ (the components take turns: same arithmetic, a third
// of the LDS, three times the barriers).
template <typename T, int N, int OP, bool SEQ = false>
__device__ __forceinline__ void xgreen3_body(cpx<T>* __restrict__ S, const Dims& d, const cpx<T>* __restrict__ tw,
                                             const WaveTables<T>& wt, const GreenConst<T>& g, cpx<T>* lds, int bx) {
  using C = LineCfg<T, N, 3>;
  const int t = threadIdx.x % C::P, l = threadIdx.x / C::P;
  const int nlines = d.Hp * d.ny;
  const int line = bx * C::LPB + l;
  int mz, my;
  const bool ok = xline_of(d, line, mz, my);
  const long long cs = (long long)nlines * N;
  cpx<T>* base = S + (long long)(ok ? line : 0) * N + t;
  cpx<T> v[3][C::E];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int m = 0; m < C::E; ++m) v[c][m] = ok ? base[c * cs + m * C::P] : mk(T(0), T(0));
  const auto at = [l](int c, int pos) { return ((SEQ ? 0 : c) * C::LPB + l) * C::LINE + C::pos(pos); };
  fft_regs<T, N, C::E, 3, false, SEQ>(v, t, lds, at, tw);
#pragma unroll
  for (int m = 0; m < C::E; ++m) {
    cpx<T> b[3] = {v[0][m], v[1][m], v[2][m]};
    green_disp<T, OP>(b, wt, t + m * C::P, my, mz, g);
#pragma unroll
    for (int c = 0; c < 3; ++c) v[c][m] = b[c];
  }
  fft_regs<T, N, C::E, 3, true, SEQ>(v, t, lds, at, tw);
  if (ok) {
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int m = 0; m < C::E; ++m) base[c * cs + m * C::P] = v[c][m];
  }
}


template <typename T, int N, int OP>
__global__ __launch_bounds__((LineCfg<T, N, 3>::NT)) void k_xgreen3(cpx<T>* __restrict__ S, Dims d,
                                                                  const cpx<T>* __restrict__ tw, WaveTables<T> wt,
                                                                  GreenConst<T> g, Batch bt,
                                                                  const GreenConst<T>* __restrict__ gs) {
  using C = LineCfg<T, N, 3>;
  if (bt.active) {
    const long long smp = bt.active[blockIdx.y];
    S += smp * 3 * spec_size(d);
    if (gs) g = gs[smp];
  }
  // the three components exchange through LDS together (51 KiB at 512):
  // a third of the barriers of taking turns
  __shared__ cpx<T> lds[3 * C::LPB * C::LINE];
  xgreen3_body<T, N, OP>(S, d, tw, wt, g, lds, blockIdx.x);
}

template <typename T, int N, int OP>
__global__ __launch_bounds__((LineCfg<T, N, 6>::NT)) void k_xgreen6(cpx<T>* __restrict__ S, Dims d,
                                                                  const cpx<T>* __restrict__ tw, WaveTables<T> wt,
                                                                  GreenConst<T> g) {
  using C = LineCfg<T, N, 6>;
  __shared__ cpx<T> lds[C::LPB * C::LINE];
  const int t = threadIdx.x % C::P, l = threadIdx.x / C::P;
  const int nlines = d.Hp * d.ny;
  const int line = blockIdx.x * C::LPB + l;
  int mz, my;
  const bool ok = xline_of(d, line, mz, my);
  const long long cs = (long long)nlines * N;
  cpx<T>* base = S + (long long)(ok ? line : 0) * N + t;
  cpx<T> v[6][C::E];
#pragma unroll
  for (int c = 0; c < 6; ++c)
#pragma unroll
    for (int m = 0; m < C::E; ++m) v[c][m] = ok ? base[c * cs + m * C::P] : mk(T(0), T(0));
  const auto at = [l](int, int pos) { return l * C::LINE + C::pos(pos); };
  fft_regs<T, N, C::E, 6, false, true>(v, t, lds, at, tw);
#pragma unroll
  for (int m = 0; m < C::E; ++m) {
    cpx<T> tv[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) tv[c] = v[c][m];
    green_six<T, OP>(tv, wt, t + m * C::P, my, mz, g);
#pragma unroll
    for (int c = 0; c < 6; ++c) v[c][m] = tv[c];
  }
  fft_regs<T, N, C::E, 6, true, true>(v, t, lds, at, tw);
  if (ok) {
#pragma unroll
    for (int c = 0; c < 6; ++c)
#pragma unroll
      for (int m = 0; m < C::E; ++m) base[c * cs + m * C::P] = v[c][m];
  }
}

// Spectral equilibrium norm (eq. (43)) of a stress whose z and y transforms
// are in S: forward x transform, then per frequency the divergence.
//   XETA_PLAIN  partial sums of |conj(k).sigma|^2 over q and its mirror;
//   XETA_BASE   the same with a stored divergence spectrum added before the
//               square (the anchor's stress, a = div sigma(delta) + A,
//               b = div of the mirror + B): eta of anchor + correction
//               without forming their sum in float32;
//   XETA_STORE  writes A and B (rounded to TS) instead of reducing.
// A and B are complex [3][Hp ny lines][nx], the spectrum's line layout
// (modes XETA_* in fe_kernels.h).

template <typename T, int N, int OP, int MODE, typename TS>
__global__ __launch_bounds__((LineCfg<T, N, 6>::NT)) void k_xeta6(const cpx<T>* __restrict__ S, Dims d,
                                                                const cpx<T>* __restrict__ tw, WaveTables<T> wt,
                                                                double* __restrict__ partials,
                                                                cpx<TS>* __restrict__ base) {
  using C = LineCfg<T, N, 6>;
  __shared__ cpx<T> lds[C::LPB * C::LINE];
  __shared__ double red[16];
  const int t = threadIdx.x % C::P, l = threadIdx.x / C::P;
  const int nlines = d.Hp * d.ny;
  const int line = blockIdx.x * C::LPB + l;
  int mz, my;
  const bool ok = xline_of(d, line, mz, my);
  const long long cs = (long long)nlines * N;
  const cpx<T>* src = S + (long long)(ok ? line : 0) * N + t;
  cpx<T> v[6][C::E];
#pragma unroll
  for (int c = 0; c < 6; ++c)
#pragma unroll
    for (int m = 0; m < C::E; ++m) v[c][m] = ok ? src[c * cs + m * C::P] : mk(T(0), T(0));
  const auto at = [l](int, int pos) { return l * C::LINE + C::pos(pos); };
  fft_regs<T, N, C::E, 6, false, true>(v, t, lds, at, tw);
  const long long bs = 3 * cs;  // B follows A
  cpx<TS>* bl = base + (long long)(ok ? line : 0) * N + t;
  double acc[1] = {0.0};
  if (ok) {
#pragma unroll
    for (int m = 0; m < C::E; ++m) {
      cpx<T> sv[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) sv[c] = v[c][m];
      if (MODE == XETA_PLAIN) {
        acc[0] += eta_six<T, OP>(sv, wt, t + m * C::P, my, mz, d);
      } else {
        cpx<T> a[3], b[3];
        const bool mirror = div_six<T, OP>(sv, wt, t + m * C::P, my, mz, d, a, b);
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          cpx<TS>* pa = bl + j * cs + m * C::P;
          cpx<TS>* pb = bl + bs + j * cs + m * C::P;
          if (MODE == XETA_STORE) {
            *pa = mk(TS(a[j].re), TS(a[j].im));
            *pb = mk(TS(b[j].re), TS(b[j].im));
          } else {
            const cpx<TS> A = *pa;
            const double ar = double(a[j].re) + double(A.re), ai = double(a[j].im) + double(A.im);
            acc[0] += ar * ar + ai * ai;
            if (mirror) {
              const cpx<TS> B = *pb;
              const double br = double(b[j].re) + double(B.re), bi = double(b[j].im) + double(B.im);
              acc[0] += br * br + bi * bi;
            }
          }
        }
      }
    }
  }
  if (MODE == XETA_STORE) return;
  block_sum<1>(acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = acc[0];
}

// ---------------------------------------------------------------------------
// length dispatch
// ---------------------------------------------------------------------------
template <class F>
static bool dispatch_length(int n, F&& f) {
  switch (n) {
#define FE_CASE(NN)                                \
  case NN:                                         \
    f(std::integral_constant<int, NN>());          \
    return true;
    FE_FOR_EACH_LENGTH(FE_CASE)
#undef FE_CASE
  }
  return false;
}
// z passes: the lengths above and 1 (one-plane cells)
template <class F>
static bool dispatch_z_length(int n, F&& f) {
  if (n == 1) {
    f(std::integral_constant<int, 1>());
    return true;
  }
  return dispatch_length(n, f);
}

template <typename T, int N>
inline int x_blocks(const Dims& d, int nc) {
  const int lpb = nc == 3 ? LineCfg<T, N, 3>::LPB : LineCfg<T, N, 6>::LPB;
  return (d.Hp * d.ny + lpb - 1) / lpb;
}

}  // namespace fe
