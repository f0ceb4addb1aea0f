// Warm-start U-Net: weight packing, input features, pooling, upsampling and
// concatenation, the linear head with its mean correction and loss, and Adam.
// Every reduction sums per-block partials in a fixed order (deterministic).
#include "fe_nn.h"

namespace fe {
namespace nn {

namespace {

inline int blocks_for(long long n, int per = 256, int cap = 1 << 20) {
  long long b = (n + per - 1) / per;
  if (b < 1) b = 1;
  return (int)(b < cap ? b : cap);
}

__device__ __forceinline__ void unpack8(const u32x4& v, float (&f)[8]) {
  const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    f[2 * i] = bf2f((uint16_t)(w[i] & 0xffffu));
    f[2 * i + 1] = bf2f((uint16_t)(w[i] >> 16));
  }
}

__device__ __forceinline__ u32x4 pack8(const float (&f)[8]) {
  u32x4 v;
  v.x = (uint32_t)f2bf(f[0]) | ((uint32_t)f2bf(f[1]) << 16);
  v.y = (uint32_t)f2bf(f[2]) | ((uint32_t)f2bf(f[3]) << 16);
  v.z = (uint32_t)f2bf(f[4]) | ((uint32_t)f2bf(f[5]) << 16);
  v.w = (uint32_t)f2bf(f[6]) | ((uint32_t)f2bf(f[7]) << 16);
  return v;
}

template <int NV>
__device__ __forceinline__ void block_sum_d(double (&a)[NV], double* red) {
  // 256 threads: wavefront reduction by shuffles, then across the 4 waves
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double v = a[i];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    a[i] = v;
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int i = 0; i < NV; ++i) red[w * NV + i] = a[i];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int i = 0; i < NV; ++i) a[i] = red[i] + red[NV + i] + red[2 * NV + i] + red[3 * NV + i];
}

}  // namespace

// ---------------------------------------------------------------------------
// weights
// ---------------------------------------------------------------------------
// Fragment of the A operand for lane (q, c): output channel o = 16 mt + c,
// reduction slots e < 8 -> tap ks TPK + 8q / CCH, input channel
// ch CCH + (8q mod CCH) + e.  flip: weights of the input-gradient convolution,
// W'[t][o'][c'] = W[26 - t][c'][o'] (input and output channels exchanged).
__global__ void k_pack(const float* __restrict__ w, int cin, int cout, int flip, u32x4* __restrict__ out) {
  const int CI = flip ? cout : cin, CO = flip ? cin : cout;
  const int CCH = conv_cch(CI), TPK = 32 / CCH, KS = conv_ksteps(CI), MT = CO / 16, NCH = CI / CCH;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= NCH * KS * MT * 64) return;
  const int lane = idx % 64;
  int rest = idx / 64;
  const int mt = rest % MT;
  rest /= MT;
  const int ks = rest % KS, ch = rest / KS;
  const int c = lane & 15, q = lane >> 4;
  // step ks = 3 gi + kk: slot (8q)/CCH takes the (dz, dx) column gi TPK + slot
  // at dy = kk - 1 (the order of the convolution kernel's register window)
  const int col = (ks / 3) * TPK + (8 * q) / CCH, kk = ks % 3;
  const int tap = col < 9 ? (col / 3) * 9 + kk * 3 + col % 3 : 27;
  const int c0 = ch * CCH + (8 * q) % CCH, o = mt * 16 + c;
  float f[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    float v = 0.f;
    if (tap < 27) v = flip ? w[((long long)(26 - tap) * cin + o) * cout + c0 + e] : w[((long long)tap * cin + c0 + e) * cout + o];
    f[e] = v;
  }
  out[idx] = pack8(f);
}

void pack_weights(const float* w, int cin, int cout, int flip, uint16_t* out, hipStream_t s) {
  const int CI = flip ? cout : cin, CO = flip ? cin : cout;
  const long long n = packed_elems(CI, CO) / 8;
  hipLaunchKernelGGL(k_pack, dim3(blocks_for(n)), dim3(256), 0, s, w, cin, cout, flip, reinterpret_cast<u32x4*>(out));
}

// ---------------------------------------------------------------------------
// input features: log10(E)/3, 10 (nu - 0.3), eps_bar
// ---------------------------------------------------------------------------
__global__ void k_features(const uint8_t* __restrict__ phase, const FeatTab* __restrict__ tabs, u32x4* __restrict__ x0,
                           Grid3 g) {
  const long long N = (long long)g.nx * g.ny * g.nz;
  const int smp = blockIdx.y;
  const FeatTab& t = tabs[smp];
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < N; v += (long long)gridDim.x * blockDim.x) {
    const int p = phase[smp * N + v];
    const float f[8] = {t.logE[p], t.nu[p], t.macro[0], t.macro[1], t.macro[2], t.macro[3], t.macro[4], t.macro[5]};
    x0[smp * N + v] = pack8(f);
  }
}

void features(const uint8_t* phase, const FeatTab* tabs, uint16_t* x0, Grid3 g, hipStream_t s) {
  const long long N = (long long)g.nx * g.ny * g.nz;
  hipLaunchKernelGGL(k_features, dim3(blocks_for(N, 256, 4096), g.nb), dim3(256), 0, s, phase, tabs,
                     reinterpret_cast<u32x4*>(x0), g);
}

// ---------------------------------------------------------------------------
// pooling, upsampling, concatenation and their gradients (8 channels per thread)
// ---------------------------------------------------------------------------
__device__ __forceinline__ long long fine_index(const Grid3& f, int smp, int z, int y, int x) {
  return (((long long)smp * f.nz + z) * f.ny + y) * f.nx + x;
}

// coarse voxel index v of the grid (nx/2, ny/2, nz/2) -> (smp, Z, Y, X)
__device__ __forceinline__ void coarse_coords(long long v, const Grid3& f, int& smp, int& Z, int& Y, int& X) {
  const int cx = f.nx / 2, cy = f.ny / 2, cz = f.nz / 2;
  X = (int)(v % cx);
  v /= cx;
  Y = (int)(v % cy);
  v /= cy;
  Z = (int)(v % cz);
  smp = (int)(v / cz);
}

__global__ void k_pool2(const u32x4* __restrict__ x, int pieces, u32x4* __restrict__ y, Grid3 f, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const int p = (int)(i % pieces);
    int smp, Z, Y, X;
    coarse_coords(i / pieces, f, smp, Z, Y, X);
    float acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      float v[8];
      unpack8(x[fine_index(f, smp, 2 * Z + (a >> 2), 2 * Y + ((a >> 1) & 1), 2 * X + (a & 1)) * pieces + p], v);
#pragma unroll
      for (int e = 0; e < 8; ++e) acc[e] += v[e];
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) acc[e] *= 0.125f;
    y[i] = pack8(acc);
  }
}

void pool2(const uint16_t* x, int c, uint16_t* y, Grid3 f, hipStream_t s) {
  const long long n = f.voxels() / 8 * (c / 8);
  hipLaunchKernelGGL(k_pool2, dim3(blocks_for(n)), dim3(256), 0, s, reinterpret_cast<const u32x4*>(x), c / 8,
                     reinterpret_cast<u32x4*>(y), f, n);
}

__global__ void k_up_concat(const u32x4* __restrict__ coarse, int pa, const u32x4* __restrict__ skip, int pb,
                            u32x4* __restrict__ out, Grid3 f, long long n) {
  const int P = pa + pb;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const int p = (int)(i % P);
    const long long v = i / P;
    if (p < pa) {
      long long r = v;
      const int x = (int)(r % f.nx);
      r /= f.nx;
      const int y = (int)(r % f.ny);
      r /= f.ny;
      const int z = (int)(r % f.nz);
      const int smp = (int)(r / f.nz);
      const long long cv = (((long long)smp * (f.nz / 2) + z / 2) * (f.ny / 2) + y / 2) * (f.nx / 2) + x / 2;
      out[i] = coarse[cv * pa + p];
    } else {
      out[i] = skip[v * pb + (p - pa)];
    }
  }
}

void up_concat(const uint16_t* coarse, int ca, const uint16_t* skip, int cb, uint16_t* out, Grid3 f, hipStream_t s) {
  const long long n = f.voxels() * ((ca + cb) / 8);
  hipLaunchKernelGGL(k_up_concat, dim3(blocks_for(n)), dim3(256), 0, s, reinterpret_cast<const u32x4*>(coarse), ca / 8,
                     reinterpret_cast<const u32x4*>(skip), cb / 8, reinterpret_cast<u32x4*>(out), f, n);
}

__global__ void k_up_backward(const u32x4* __restrict__ gcat, int pa, int pb, u32x4* __restrict__ gc, Grid3 f,
                              long long n) {
  const int P = pa + pb;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const int p = (int)(i % pa);
    int smp, Z, Y, X;
    coarse_coords(i / pa, f, smp, Z, Y, X);
    float acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      float v[8];
      unpack8(gcat[fine_index(f, smp, 2 * Z + (a >> 2), 2 * Y + ((a >> 1) & 1), 2 * X + (a & 1)) * P + p], v);
#pragma unroll
      for (int e = 0; e < 8; ++e) acc[e] += v[e];
    }
    gc[i] = pack8(acc);
  }
}

void up_backward(const uint16_t* gcat, int ca, int cb, uint16_t* gcoarse, Grid3 f, hipStream_t s) {
  const long long n = f.voxels() / 8 * (ca / 8);
  hipLaunchKernelGGL(k_up_backward, dim3(blocks_for(n)), dim3(256), 0, s, reinterpret_cast<const u32x4*>(gcat), ca / 8,
                     cb / 8, reinterpret_cast<u32x4*>(gcoarse), f, n);
}

__global__ void k_pool_backward_add(const u32x4* __restrict__ gpool, const u32x4* __restrict__ gcat, int pa, int pc,
                                    u32x4* __restrict__ g, Grid3 f, long long n) {
  const int P = pa + pc;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const int p = (int)(i % pc);
    const long long v = i / pc;
    long long r = v;
    const int x = (int)(r % f.nx);
    r /= f.nx;
    const int y = (int)(r % f.ny);
    r /= f.ny;
    const int z = (int)(r % f.nz);
    const int smp = (int)(r / f.nz);
    const long long cv = (((long long)smp * (f.nz / 2) + z / 2) * (f.ny / 2) + y / 2) * (f.nx / 2) + x / 2;
    float a[8], b[8];
    unpack8(gpool[cv * pc + p], a);
    unpack8(gcat[v * P + pa + p], b);
#pragma unroll
    for (int e = 0; e < 8; ++e) a[e] = a[e] * 0.125f + b[e];
    g[i] = pack8(a);
  }
}

void pool_backward_add(const uint16_t* gpool, const uint16_t* gcat, int ca, int c, uint16_t* g, Grid3 f,
                       hipStream_t s) {
  const long long n = f.voxels() * (c / 8);
  hipLaunchKernelGGL(k_pool_backward_add, dim3(blocks_for(n)), dim3(256), 0, s, reinterpret_cast<const u32x4*>(gpool),
                     reinterpret_cast<const u32x4*>(gcat), ca / 8, c / 8, reinterpret_cast<u32x4*>(g), f, n);
}

// ---------------------------------------------------------------------------
// bias gradient: db[c] = sum_v dy[v, c] (ymask[v, c] > 0)
// ---------------------------------------------------------------------------
constexpr int kBiasBlocks = 512;

__global__ __launch_bounds__(256) void k_bias_partials(const uint16_t* __restrict__ dy, const uint16_t* __restrict__ ym,
                                                       int c, long long V, float* __restrict__ partials) {
  __shared__ float red[256];
  const int per = 256 / c;  // voxels per pass (c divides 256)
  const int ch = threadIdx.x % c, vo = threadIdx.x / c;
  float acc = 0.f;
  if (vo < per)
    for (long long v = blockIdx.x * (long long)per + vo; v < V; v += (long long)gridDim.x * per) {
      const uint16_t d = dy[v * c + ch];
      bool keep = true;
      if (ym) {
        const uint16_t m = ym[v * c + ch];
        keep = m != 0 && !(m & 0x8000u);
      }
      if (keep) acc += bf2f(d);
    }
  red[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x < c) {
    float s = 0.f;
    for (int k = 0; k < per; ++k) s += red[k * c + threadIdx.x];
    partials[blockIdx.x * c + threadIdx.x] = s;
  }
}

// one workgroup of 256 per channel: thread t adds rows t, t + 256, ..., then
// the fixed-order tree in float64
__global__ __launch_bounds__(256) void k_bias_reduce(const float* __restrict__ partials, int nb, int c,
                                                     float* __restrict__ db) {
  __shared__ double red[4];
  const int ch = blockIdx.x;
  double acc[1] = {0.0};
  for (int b = threadIdx.x; b < nb; b += blockDim.x) acc[0] += (double)partials[b * c + ch];
  block_sum_d<1>(acc, red);
  if (threadIdx.x == 0) db[ch] = (float)acc[0];
}

int bias_grad(const uint16_t* dy, const uint16_t* ymask, int c, float* partials, float* db, Grid3 g, hipStream_t s) {
  const long long V = g.voxels();
  long long nb = (V + (256 / c) - 1) / (256 / c);
  if (nb > kBiasBlocks) nb = kBiasBlocks;
  hipLaunchKernelGGL(k_bias_partials, dim3((int)nb), dim3(256), 0, s, dy, ymask, c, V, partials);
  hipLaunchKernelGGL(k_bias_reduce, dim3(c), dim3(256), 0, s, partials, (int)nb, c, db);
  return (int)nb;
}

// ---------------------------------------------------------------------------
// head (16 -> 6, linear), mean correction, loss
// ---------------------------------------------------------------------------
// Blocks per sample of the head kernels: about 2048 in all (a single 512^3
// prediction needs the whole chip), 64 to 1024 per sample, never more than
// the sample's voxels fill.
int head_blocks(Grid3 g) {
  const long long N = (long long)g.nx * g.ny * g.nz;
  int b = 2048 / (g.nb > 0 ? g.nb : 1);
  b = b < 64 ? 64 : (b > 1024 ? 1024 : b);
  const long long fill = (N + 255) / 256;
  return (int)(b > fill ? fill : b);
}

__device__ __forceinline__ void head_eval(const u32x4* __restrict__ d1, long long v, const float* __restrict__ hw,
                                          const float* __restrict__ hb, float (&x)[16], float (&p)[6]) {
  float a[8], b[8];
  unpack8(d1[2 * v], a);
  unpack8(d1[2 * v + 1], b);
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    x[e] = a[e];
    x[8 + e] = b[e];
  }
#pragma unroll
  for (int o = 0; o < 6; ++o) {
    float s = hb[o];
#pragma unroll
    for (int c = 0; c < 16; ++c) s += x[c] * hw[c * 6 + o];
    p[o] = s;
  }
}

__device__ __forceinline__ float load_target(const void* t, int is_bf16, long long i) {
  return is_bf16 ? bf2f(static_cast<const uint16_t*>(t)[i]) : static_cast<const float*>(t)[i];
}

// partials[smp][block][12]: sums of p (6) and of the target (6)
__global__ __launch_bounds__(256) void k_head_stats(const u32x4* __restrict__ d1, const float* __restrict__ hw,
                                                    const float* __restrict__ hb, const void* target, int tbf16,
                                                    double* __restrict__ partials, Grid3 g) {
  __shared__ double red[4 * 12];
  const long long N = (long long)g.nx * g.ny * g.nz;
  const int smp = blockIdx.y;
  double acc[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < N; v += (long long)gridDim.x * blockDim.x) {
    float x[16], p[6];
    head_eval(d1, smp * N + v, hw, hb, x, p);
#pragma unroll
    for (int o = 0; o < 6; ++o) acc[o] += p[o];
    if (target)
#pragma unroll
      for (int o = 0; o < 6; ++o) acc[6 + o] += load_target(target, tbf16, (smp * 6LL + o) * N + v);
  }
  block_sum_d<12>(acc, red);
  if (threadIdx.x == 0)
    for (int i = 0; i < 12; ++i) partials[((long long)smp * gridDim.x + blockIdx.x) * 12 + i] = acc[i];
}

// one workgroup of 256 per sample: thread t adds records t, t + 256, ...,
// then the fixed-order tree (one thread walking all records waited out one
// load latency per record)
__global__ __launch_bounds__(256) void k_head_sums(const double* __restrict__ partials, int nblk,
                                                   double* __restrict__ sums) {
  __shared__ double red[4 * 12];
  const int smp = blockIdx.x;
  double acc[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < nblk; b += blockDim.x)
#pragma unroll
    for (int i = 0; i < 12; ++i) acc[i] += partials[((long long)smp * nblk + b) * 12 + i];
  block_sum_d<12>(acc, red);
  if (threadIdx.x == 0)
    for (int i = 0; i < 12; ++i) sums[smp * 12 + i] = acc[i];
}

int head_stats(const uint16_t* d1, const float* hw, const float* hb, const void* target, int target_bf16,
               double* partials, double* sums, Grid3 g, hipStream_t s) {
  const int hb_n = head_blocks(g);
  hipLaunchKernelGGL(k_head_stats, dim3(hb_n, g.nb), dim3(256), 0, s, reinterpret_cast<const u32x4*>(d1), hw, hb,
                     target, target_bf16, partials, g);
  hipLaunchKernelGGL(k_head_sums, dim3(g.nb), dim3(256), 0, s, partials, hb_n, sums);
  return hb_n;
}

__global__ void k_head_predict(const u32x4* __restrict__ d1, const float* __restrict__ hw, const float* __restrict__ hb,
                               const double* __restrict__ sums, const FeatTab* __restrict__ tabs, float* __restrict__ out,
                               Grid3 g) {
  const long long N = (long long)g.nx * g.ny * g.nz;
  const int smp = blockIdx.y;
  float shift[6];
#pragma unroll
  for (int o = 0; o < 6; ++o) shift[o] = (float)((double)tabs[smp].macro[o] - sums[smp * 12 + o] / (double)N);
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < N; v += (long long)gridDim.x * blockDim.x) {
    float x[16], p[6];
    head_eval(d1, smp * N + v, hw, hb, x, p);
#pragma unroll
    for (int o = 0; o < 6; ++o) out[(smp * 6LL + o) * N + v] = p[o] + shift[o];
  }
}

void head_predict(const uint16_t* d1, const float* hw, const float* hb, const double* sums, const FeatTab* tabs,
                  float* out, Grid3 g, hipStream_t s) {
  const long long N = (long long)g.nx * g.ny * g.nz;
  hipLaunchKernelGGL(k_head_predict, dim3(blocks_for(N, 256, 4096), g.nb), dim3(256), 0, s,
                     reinterpret_cast<const u32x4*>(d1), hw, hb, sums, tabs, out, g);
}

// Training: gp = 2/(B 6 N) (diff - mean_v diff), diff = p - mean(p) + eps_bar - target,
// where mean_v diff = eps_bar - mean(target) (the mean of p - mean(p) is zero).
// Writes gd1 = gp hw^T (bf16) and per-block partials: loss (1), head weight
// gradient (96), head bias gradient (6).
constexpr int kHeadNV = 1 + 96 + 6;

__global__ __launch_bounds__(256) void k_head_backward(const u32x4* __restrict__ d1, const float* __restrict__ hw,
                                                       const float* __restrict__ hb, const double* __restrict__ sums,
                                                       const FeatTab* __restrict__ tabs, const void* target, int tbf16,
                                                       u32x4* __restrict__ gd1, double* __restrict__ partials,
                                                       Grid3 g) {
  __shared__ double red[4 * 8];
  const long long N = (long long)g.nx * g.ny * g.nz;
  const int smp = blockIdx.y;
  const double inv = 1.0 / (double)N;
  const float scale = (float)(2.0 / ((double)g.nb * 6.0 * (double)N));
  float shift[6], mdiff[6];
#pragma unroll
  for (int o = 0; o < 6; ++o) {
    const double mac = (double)tabs[smp].macro[o];
    shift[o] = (float)(mac - sums[smp * 12 + o] * inv);
    mdiff[o] = (float)(mac - sums[smp * 12 + 6 + o] * inv);
  }
  double loss = 0.0;
  float gw[96], gb[6];
#pragma unroll
  for (int i = 0; i < 96; ++i) gw[i] = 0.f;
#pragma unroll
  for (int o = 0; o < 6; ++o) gb[o] = 0.f;
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < N; v += (long long)gridDim.x * blockDim.x) {
    float x[16], p[6], gp[6];
    head_eval(d1, smp * N + v, hw, hb, x, p);
#pragma unroll
    for (int o = 0; o < 6; ++o) {
      const float diff = p[o] + shift[o] - load_target(target, tbf16, (smp * 6LL + o) * N + v);
      loss += (double)diff * (double)diff;
      gp[o] = scale * (diff - mdiff[o]);
      gb[o] += gp[o];
    }
    float gx[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      float s = 0.f;
#pragma unroll
      for (int o = 0; o < 6; ++o) {
        s += gp[o] * hw[c * 6 + o];
        gw[c * 6 + o] += x[c] * gp[o];
      }
      gx[c] = s;
    }
    float lo[8], hi[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      lo[e] = gx[e];
      hi[e] = gx[8 + e];
    }
    gd1[2 * (smp * N + v)] = pack8(lo);
    gd1[2 * (smp * N + v) + 1] = pack8(hi);
  }
  // block sums in chunks of 8 values
  double* out = partials + ((long long)smp * gridDim.x + blockIdx.x) * kHeadNV;
  {
    double a[8] = {loss, 0, 0, 0, 0, 0, 0, 0};
    block_sum_d<8>(a, red);
    if (threadIdx.x == 0) out[0] = a[0];
    __syncthreads();
  }
  for (int c0 = 0; c0 < 96; c0 += 8) {
    double a[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) a[e] = gw[c0 + e];
    block_sum_d<8>(a, red);
    if (threadIdx.x == 0)
      for (int e = 0; e < 8; ++e) out[1 + c0 + e] = a[e];
    __syncthreads();
  }
  {
    double a[8] = {gb[0], gb[1], gb[2], gb[3], gb[4], gb[5], 0, 0};
    block_sum_d<8>(a, red);
    if (threadIdx.x == 0)
      for (int e = 0; e < 6; ++e) out[97 + e] = a[e];
  }
}

// one workgroup of 256 per value: thread t adds rows t, t + 256, ..., then
// the fixed-order tree
__global__ __launch_bounds__(256) void k_head_backward_reduce(const double* __restrict__ partials, int nrows,
                                                              double* __restrict__ loss_out, float* __restrict__ ghw,
                                                              float* __restrict__ ghb, double loss_scale) {
  __shared__ double red[4];
  const int i = blockIdx.x;
  double acc[1] = {0.0};
  for (int r = threadIdx.x; r < nrows; r += blockDim.x) acc[0] += partials[(long long)r * kHeadNV + i];
  block_sum_d<1>(acc, red);
  if (threadIdx.x != 0) return;
  const double s = acc[0];
  if (i == 0)
    *loss_out = s * loss_scale;
  else if (i <= 96)
    ghw[i - 1] = (float)s;
  else
    ghb[i - 97] = (float)s;
}

int head_backward(const uint16_t* d1, const float* hw, const float* hb, const double* sums, const FeatTab* tabs,
                  const void* target, int target_bf16, uint16_t* gd1, double* partials, double* out_loss, float* ghw,
                  float* ghb, Grid3 g, hipStream_t s) {
  const int hb_n = head_blocks(g);
  hipLaunchKernelGGL(k_head_backward, dim3(hb_n, g.nb), dim3(256), 0, s, reinterpret_cast<const u32x4*>(d1), hw,
                     hb, sums, tabs, target, target_bf16, reinterpret_cast<u32x4*>(gd1), partials, g);
  const double scale = 1.0 / ((double)g.nb * 6.0 * (double)g.nx * g.ny * g.nz);
  hipLaunchKernelGGL(k_head_backward_reduce, dim3(kHeadNV), dim3(256), 0, s, partials, hb_n * g.nb, out_loss, ghw,
                     ghb, scale);
  return hb_n;
}

// ---------------------------------------------------------------------------
// Adam (bias-corrected moments), float32 master weights
// ---------------------------------------------------------------------------
__global__ void k_adam(float* __restrict__ th, const float* __restrict__ gr, float* __restrict__ m, float* __restrict__ v,
                       long long n, float lr, float b1, float b2, float eps, float c1, float c2) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const float g = gr[i];
    const float mi = b1 * m[i] + (1.f - b1) * g;
    const float vi = b2 * v[i] + (1.f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    th[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
  }
}

void adam(float* theta, const float* grad, float* m, float* v, long long n, float lr, float b1, float b2, float eps,
          int t, hipStream_t s) {
  const float c1 = (float)(1.0 / (1.0 - std::pow((double)b1, t)));
  const float c2 = (float)(1.0 / (1.0 - std::pow((double)b2, t)));
  hipLaunchKernelGGL(k_adam, dim3(blocks_for(n, 256, 8192)), dim3(256), 0, s, theta, grad, m, v, n, lr, b1, b2, eps, c1,
                     c2);
}

}  // namespace nn
}  // namespace fe
