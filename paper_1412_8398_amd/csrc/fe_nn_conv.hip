// 3^3 periodic convolutions of the warm-start U-Net on the gfx950 matrix cores
// (v_mfma_f32_16x16x32_bf16: bf16 operands, fp32 accumulation).
//
// Operand layout of one 16x16x32 product (wavefront of 64 lanes, lane l,
// group q = l / 16, column c = l % 16):
//   A[i = c][k = 8q + e], B[k = 8q + e][j = c] for e < 8 (16 bytes per lane),
//   D[4q + r][c] for r < 4.
// Forward / input-gradient: i = output channel, j = voxel along x, k = (tap,
// input channel).  Weight gradient: i = output channel, j = input channel,
// k = voxel.
#include "fe_nn.h"

namespace fe {
namespace nn {

__device__ __forceinline__ int wrapi(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

// keep the 16-bit halves of v whose mask half is a positive bf16
__device__ __forceinline__ uint32_t mask2(uint32_t v, uint32_t m) {
  const uint32_t lo = m & 0xffffu, hi = m >> 16;
  uint32_t r = 0;
  if (lo != 0u && !(lo & 0x8000u)) r |= v & 0xffffu;
  if (hi != 0u && !(hi & 0x8000u)) r |= v & 0xffff0000u;
  return r;
}

__device__ __forceinline__ u32x4 mask8(u32x4 v, u32x4 m) {
  v.x = mask2(v.x, m.x);
  v.y = mask2(v.y, m.y);
  v.z = mask2(v.z, m.z);
  v.w = mask2(v.w, m.w);
  return v;
}

__device__ __forceinline__ f32x4 mfma(u32x4 a, u32x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0,
                                                  0, 0);
}

struct TileCoord {
  int x0, y0, z0, smp;
};

__device__ __forceinline__ TileCoord tile_of(int t, const Grid3& g) {
  const int ntx = (g.nx + TX - 1) / TX, nty = (g.ny + TY - 1) / TY, ntz = (g.nz + TZ - 1) / TZ;
  TileCoord c;
  c.x0 = (t % ntx) * TX;
  t /= ntx;
  c.y0 = (t % nty) * TY;
  t /= nty;
  c.z0 = (t % ntz) * TZ;
  c.smp = t / ntz;
  return c;
}

// ---------------------------------------------------------------------------
// forward (and input gradient with flipped, transposed weights)
// ---------------------------------------------------------------------------
// With CA > 0 the input is the concatenation [nearest upsampling of XC
// (CA channels on the grid halved in each direction), X (CIN - CA channels)]
// read in place: a decoder layer without its concatenated input in HBM (the
// channel chunks never straddle the two sources, CA being a multiple of CCH).
template <int CIN, int COUT, bool RELU, bool MASKED, int CA = 0>
__global__ __launch_bounds__(256) void k_conv3(const uint16_t* __restrict__ X, const uint16_t* __restrict__ M,
                                               const u32x4* __restrict__ W, const float* __restrict__ bias,
                                               uint16_t* __restrict__ Y, Grid3 g,
                                               const uint16_t* __restrict__ XC = nullptr) {
  constexpr int CCH = conv_cch(CIN), NCH = CIN / CCH, TPK = 32 / CCH, KS = conv_ksteps(CIN), MT = COUT / 16;
  constexpr int NG = conv_groups(CIN);
  constexpr int PIECES = CCH / 8;
  __shared__ u32x4 lds[HV * PIECES];  // [halo voxel][8-channel piece]
  const TileCoord tc = tile_of(blockIdx.x, g);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int j = lane & 15, grp = lane >> 4;
  const long long zb = (long long)tc.smp * g.nz;
  f32x4 acc[MT][TY];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int r = 0; r < TY; ++r) acc[mt][r] = f32x4{0.f, 0.f, 0.f, 0.f};

  // this lane's reduction group: tap slot within the k step and channel piece
  const int slot = (grp * 8) / CCH, pc = ((grp * 8) % CCH) / 8;

  static_assert(CA % CCH == 0 && CA < CIN, "channel chunks within one source");
  static_assert(!(MASKED && CA > 0), "masked inputs come from one source");
  static_assert(TX % 2 == 0 && TY % 2 == 0 && TZ % 2 == 0, "tile origins even (coarse halo offsets)");
  // the tile's halo lies inside the grid (no periodic wrap): uniform
  const bool interior = tc.x0 >= 1 && tc.x0 - 1 + HX <= g.nx && tc.y0 >= 1 && tc.y0 - 1 + HY <= g.ny &&
                        tc.z0 >= 1 && tc.z0 - 1 + HZ <= g.nz;
  for (int ch = 0; ch < NCH; ++ch) {
    if (ch) __syncthreads();
    const bool from_coarse = CA > 0 && ch * CCH < CA;
    // Layers with at most 32 output channels have their halo loads in flight
    // together before the first LDS store (a load-store pair per step waits
    // out the memory latency once per step); the spare lanes of the last step
    // re-read the last halo vector, so that no load sits under a branch, and
    // the source test, uniform over the chunk, leaves each loop only its own
    // addresses.  Wider layers, and the in-place decoder layer with 32-channel
    // chunks, keep one load and store per step: the registers of the batched
    // loads cost them occupancy (measured).
    constexpr int NS = (HV * PIECES + 255) / 256;
    constexpr bool BATCHED = MT <= 2 && !(CA > 0 && CCH == 32);
    auto halo = [&](int i, int& p, int& gx, int& gy, int& gz) {
      p = i % PIECES;
      const int hv = i / PIECES;
      const int hx = hv % HX, hy = (hv / HX) % HY, hz = hv / (HX * HY);
      gx = wrapi(tc.x0 - 1 + hx, g.nx);
      gy = wrapi(tc.y0 - 1 + hy, g.ny);
      gz = wrapi(tc.z0 - 1 + hz, g.nz);
    };
    auto coarse_at = [&](int p, int gx, int gy, int gz) {
      const long long cv = (((long long)tc.smp * (g.nz / 2) + gz / 2) * (g.ny / 2) + gy / 2) * (g.nx / 2) + gx / 2;
      return *reinterpret_cast<const u32x4*>(XC + cv * CA + ch * CCH + p * 8);
    };
    auto fine_at = [&](int p, int gx, int gy, int gz) {
      const long long off = (((zb + gz) * g.ny + gy) * g.nx + gx) * (CIN - CA) + (ch * CCH - CA) + p * 8;
      u32x4 v = *reinterpret_cast<const u32x4*>(X + off);
      if (MASKED) v = mask8(v, *reinterpret_cast<const u32x4*>(M + off));
      return v;
    };
    if (BATCHED && interior) {
      // halo inside the grid: no periodic wrap, each address a uniform base
      // plus a 32-bit offset (the general path's integer divisions and 64-bit
      // products made the staging outweigh the products in issue slots)
      u32x4 st[NS];
      if (from_coarse) {
        const int cnx = g.nx / 2, cny = g.ny / 2;
        const long long cb = (((long long)tc.smp * (g.nz / 2) + tc.z0 / 2) * cny + tc.y0 / 2) * cnx + tc.x0 / 2;
#pragma unroll
        for (int q = 0; q < NS; ++q) {
          const int i = min(threadIdx.x + q * 256, HV * PIECES - 1);
          const int p = i % PIECES, hv = i / PIECES;
          const int hx = hv % HX, hy = (hv / HX) % HY, hz = hv / (HX * HY);
          // gz = z0 - 1 + hz with z0 even: gz / 2 = z0 / 2 + floor((hz - 1) / 2)
          const int lc = (((hz - 1) >> 1) * cny + ((hy - 1) >> 1)) * cnx + ((hx - 1) >> 1);
          st[q] = *reinterpret_cast<const u32x4*>(XC + (cb + lc) * CA + ch * CCH + p * 8);
        }
      } else {
        const long long fb = ((zb + tc.z0 - 1) * g.ny + (tc.y0 - 1)) * (long long)g.nx + (tc.x0 - 1);
#pragma unroll
        for (int q = 0; q < NS; ++q) {
          const int i = min(threadIdx.x + q * 256, HV * PIECES - 1);
          const int p = i % PIECES, hv = i / PIECES;
          const int hx = hv % HX, hy = (hv / HX) % HY, hz = hv / (HX * HY);
          const long long off = (fb + (hz * g.ny + hy) * g.nx + hx) * (CIN - CA) + (ch * CCH - CA) + p * 8;
          st[q] = *reinterpret_cast<const u32x4*>(X + off);
          if (MASKED) st[q] = mask8(st[q], *reinterpret_cast<const u32x4*>(M + off));
        }
      }
#pragma unroll
      for (int q = 0; q < NS; ++q) {
        const int i = threadIdx.x + q * 256;
        if (i < HV * PIECES) lds[i] = st[q];
      }
    } else if (BATCHED) {
      u32x4 st[NS];
      if (from_coarse) {
#pragma unroll
        for (int q = 0; q < NS; ++q) {
          int p, gx, gy, gz;
          halo(min(threadIdx.x + q * 256, HV * PIECES - 1), p, gx, gy, gz);
          st[q] = coarse_at(p, gx, gy, gz);
        }
      } else {
#pragma unroll
        for (int q = 0; q < NS; ++q) {
          int p, gx, gy, gz;
          halo(min(threadIdx.x + q * 256, HV * PIECES - 1), p, gx, gy, gz);
          st[q] = fine_at(p, gx, gy, gz);
        }
      }
#pragma unroll
      for (int q = 0; q < NS; ++q) {
        const int i = threadIdx.x + q * 256;
        if (i < HV * PIECES) lds[i] = st[q];
      }
    } else {
      for (int i = threadIdx.x; i < HV * PIECES; i += 256) {
        int p, gx, gy, gz;
        halo(i, p, gx, gy, gz);
        lds[i] = from_coarse ? coarse_at(p, gx, gy, gz) : fine_at(p, gx, gy, gz);
      }
    }
    __syncthreads();
    for (int gi = 0; gi < NG; ++gi) {
      int col = gi * TPK + slot;  // (dz, dx) column of this lane's taps
      if (col > 8) col = 4;       // padding slot: zero weights, any finite input
      const int dz = col / 3 - 1, dx = col % 3 - 1;
      // halo rows 0 .. TY+1 of this column: output row r, dy = kk - 1 reads row r + kk
      u32x4 fr[TY + 2];
#pragma unroll
      for (int rr = 0; rr < TY + 2; ++rr) fr[rr] = lds[(((w + dz + 1) * HY + rr) * HX + (j + dx + 1)) * PIECES + pc];
#pragma unroll
      for (int kk = 0; kk < 3; ++kk) {
        const u32x4* wp = W + (long long)(ch * KS + 3 * gi + kk) * MT * 64 + lane;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const u32x4 a = wp[mt * 64];
#pragma unroll
          for (int r = 0; r < TY; ++r) acc[mt][r] = mfma(a, fr[r + kk], acc[mt][r]);
        }
      }
    }
  }

  const int x = tc.x0 + j, z = tc.z0 + w;
  if (x >= g.nx || z >= g.nz) return;
#pragma unroll
  for (int r = 0; r < TY; ++r) {
    const int y = tc.y0 + r;
    if (y >= g.ny) continue;
    const long long vox = ((zb + z) * g.ny + y) * g.nx + x;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const int co = mt * 16 + 4 * grp;
      float o[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        o[e] = acc[mt][r][e] + (bias ? bias[co + e] : 0.f);
        if (RELU) o[e] = fmaxf(o[e], 0.f);
      }
      uint2 pk;
      pk.x = (uint32_t)f2bf(o[0]) | ((uint32_t)f2bf(o[1]) << 16);
      pk.y = (uint32_t)f2bf(o[2]) | ((uint32_t)f2bf(o[3]) << 16);
      *reinterpret_cast<uint2*>(Y + vox * COUT + co) = pk;
    }
  }
}

// ---------------------------------------------------------------------------
// weight gradient: partial sums over the tiles a block visits
// ---------------------------------------------------------------------------
template <int CIN, int COUT>
__global__ __launch_bounds__(256) void k_wgrad(const uint16_t* __restrict__ X, const uint16_t* __restrict__ DY,
                                               const uint16_t* __restrict__ YM, f32x4* __restrict__ partials,
                                               Grid3 g) {
  constexpr int CB = CIN < 16 ? CIN : 16;  // input channels per block of the product
  constexpr int NOB = COUT / 16;
  const int pair = blockIdx.y;
  const int cib = pair / NOB, cob = pair % NOB;
  __shared__ uint16_t lx[HV * 16];          // input halo, 16 channels (zero above CB)
  __shared__ uint16_t lg[TX * TY * TZ * 16];  // masked output gradient, 16 channels
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int j = lane & 15, grp = lane >> 4;
  f32x4 acc[27];
#pragma unroll
  for (int t = 0; t < 27; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int ntiles = conv_tiles(g);
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const TileCoord tc = tile_of(t, g);
    const long long zb = (long long)tc.smp * g.nz;
    __syncthreads();
    for (int i = threadIdx.x; i < HV * 2; i += 256) {
      const int p = i & 1, hv = i >> 1;
      const int hx = hv % HX, hy = (hv / HX) % HY, hz = hv / (HX * HY);
      u32x4 v = u32x4{0u, 0u, 0u, 0u};
      if (p * 8 < CB) {
        const int gx = wrapi(tc.x0 - 1 + hx, g.nx), gy = wrapi(tc.y0 - 1 + hy, g.ny),
                  gz = wrapi(tc.z0 - 1 + hz, g.nz);
        v = *reinterpret_cast<const u32x4*>(X + (((zb + gz) * g.ny + gy) * g.nx + gx) * CIN + cib * CB + p * 8);
      }
      *reinterpret_cast<u32x4*>(lx + hv * 16 + p * 8) = v;
    }
    for (int i = threadIdx.x; i < TX * TY * TZ * 2; i += 256) {
      const int p = i & 1, v = i >> 1;
      const int x = tc.x0 + (v % TX), y = tc.y0 + (v / TX) % TY, z = tc.z0 + v / (TX * TY);
      u32x4 d = u32x4{0u, 0u, 0u, 0u};
      if (x < g.nx && y < g.ny && z < g.nz) {
        const long long off = (((zb + z) * g.ny + y) * g.nx + x) * COUT + cob * 16 + p * 8;
        d = *reinterpret_cast<const u32x4*>(DY + off);
        if (YM) d = mask8(d, *reinterpret_cast<const u32x4*>(YM + off));
      }
      *reinterpret_cast<u32x4*>(lg + v * 16 + p * 8) = d;
    }
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int row = 2 * h + (grp >> 1), xb = 8 * (grp & 1);
      uint16_t av[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) av[e] = lg[((w * TY + row) * TX + xb + e) * 16 + j];
      u32x4 a;
      a.x = av[0] | ((uint32_t)av[1] << 16);
      a.y = av[2] | ((uint32_t)av[3] << 16);
      a.z = av[4] | ((uint32_t)av[5] << 16);
      a.w = av[6] | ((uint32_t)av[7] << 16);
#pragma unroll
      for (int tap = 0; tap < 27; ++tap) {
        const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
        const int base = ((w + dz + 1) * HY + (row + dy + 1)) * HX + xb + dx + 1;
        uint16_t bv[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) bv[e] = lx[(base + e) * 16 + j];
        u32x4 b;
        b.x = bv[0] | ((uint32_t)bv[1] << 16);
        b.y = bv[2] | ((uint32_t)bv[3] << 16);
        b.z = bv[4] | ((uint32_t)bv[5] << 16);
        b.w = bv[6] | ((uint32_t)bv[7] << 16);
        acc[tap] = mfma(a, b, acc[tap]);
      }
    }
  }
  f32x4* out = partials + ((long long)(pair * gridDim.x + blockIdx.x) * 4 + w) * 27 * 64;
#pragma unroll
  for (int tap = 0; tap < 27; ++tap) out[tap * 64 + lane] = acc[tap];
}

// dw[t][c][o] = fixed-order sum over the partial sets: one workgroup per
// (channel pair, tap), its 16 wavefronts each adding every 16th set for the
// 64 lanes, then the 16 slice sums in order (one thread per lane walking all
// sets waited out a load latency per set)
constexpr int kWgradSlices = 16;
template <int CIN, int COUT>
__global__ __launch_bounds__(64 * kWgradSlices) void k_wgrad_reduce(const f32x4* __restrict__ partials, int nsets,
                                                                     float* __restrict__ dw) {
  constexpr int CB = CIN < 16 ? CIN : 16;
  constexpr int NOB = COUT / 16;
  __shared__ f32x4 red[kWgradSlices][64];
  const int tap = blockIdx.x % 27, pair = blockIdx.x / 27;
  const int lane = threadIdx.x & 63, sl = threadIdx.x >> 6;
  f32x4 s = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int k = sl; k < nsets; k += kWgradSlices) s += partials[((long long)(pair * nsets + k) * 27 + tap) * 64 + lane];
  red[sl][lane] = s;
  __syncthreads();
  if (sl != 0) return;
  s = red[0][lane];
#pragma unroll
  for (int q = 1; q < kWgradSlices; ++q) s += red[q][lane];
  const int cib = pair / NOB, cob = pair % NOB;
  const int j = lane & 15, grp = lane >> 4;
  if (j >= CB) return;
  const int ci = cib * CB + j;
#pragma unroll
  for (int r = 0; r < 4; ++r) dw[((long long)tap * CIN + ci) * COUT + cob * 16 + 4 * grp + r] = s[r];
}

// ---------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------
#define FE_NN_CONV_SHAPES(X)                                                                                   \
  X(8, 16) X(16, 16) X(16, 32) X(32, 32) X(32, 64) X(64, 64) X(64, 128) X(128, 128) X(192, 64) X(96, 32)      \
      X(48, 16)
// input-gradient shapes (c_out -> c_in of the forward layers after the first)
#define FE_NN_BWD_SHAPES(X) X(16, 16) X(32, 16) X(32, 32) X(64, 32) X(64, 64) X(128, 64) X(128, 128) X(64, 192) \
  X(32, 96) X(16, 48)

bool conv_supported(int cin, int cout) {
#define FE_CASE(a, b) \
  if (cin == a && cout == b) return true;
  FE_NN_CONV_SHAPES(FE_CASE)
  FE_NN_BWD_SHAPES(FE_CASE)
#undef FE_CASE
  return false;
}

void conv3_forward(int cin, int cout, const uint16_t* x, const uint16_t* mask, const uint16_t* wpack,
                   const float* bias, int relu, uint16_t* y, Grid3 g, hipStream_t s) {
  const dim3 grid(conv_tiles(g)), block(256);
  const u32x4* wp = reinterpret_cast<const u32x4*>(wpack);
#define FE_CASE(a, b)                                                                                       \
  if (cin == a && cout == b) {                                                                              \
    if (mask)                                                                                               \
      hipLaunchKernelGGL((k_conv3<a, b, false, true>), grid, block, 0, s, x, mask, wp, bias, y, g);         \
    else if (relu)                                                                                          \
      hipLaunchKernelGGL((k_conv3<a, b, true, false>), grid, block, 0, s, x, mask, wp, bias, y, g);         \
    else                                                                                                    \
      hipLaunchKernelGGL((k_conv3<a, b, false, false>), grid, block, 0, s, x, mask, wp, bias, y, g);        \
    return;                                                                                                 \
  }
  FE_NN_CONV_SHAPES(FE_CASE)
  FE_NN_BWD_SHAPES(FE_CASE)
#undef FE_CASE
}

// the decoder layers: (c_in, c_out, coarse channels of c_in)
#define FE_NN_CAT_SHAPES(X) X(48, 16, 32) X(96, 32, 64) X(192, 64, 128)

bool conv_cat_supported(int cin, int cout, int ca) {
#define FE_CASE(a, b, c) \
  if (cin == a && cout == b && ca == c) return true;
  FE_NN_CAT_SHAPES(FE_CASE)
#undef FE_CASE
  return false;
}

void conv3_forward_cat(int cin, int cout, int ca, const uint16_t* coarse, const uint16_t* skip, const uint16_t* wpack,
                       const float* bias, int relu, uint16_t* y, Grid3 g, hipStream_t s) {
  const dim3 grid(conv_tiles(g)), block(256);
  const u32x4* wp = reinterpret_cast<const u32x4*>(wpack);
#define FE_CASE(a, b, c)                                                                                          \
  if (cin == a && cout == b && ca == c) {                                                                         \
    if (relu)                                                                                                     \
      hipLaunchKernelGGL((k_conv3<a, b, true, false, c>), grid, block, 0, s, skip, nullptr, wp, bias, y, g, coarse); \
    else                                                                                                          \
      hipLaunchKernelGGL((k_conv3<a, b, false, false, c>), grid, block, 0, s, skip, nullptr, wp, bias, y, g,      \
                         coarse);                                                                                 \
    return;                                                                                                       \
  }
  FE_NN_CAT_SHAPES(FE_CASE)
#undef FE_CASE
}

static int wgrad_blocks(int cin, int cout, const Grid3& g) {
  const int pairs = (cin < 16 ? 1 : cin / 16) * (cout / 16);
  int nb = 512 / pairs;
  if (nb < 1) nb = 1;
  const int nt = conv_tiles(g);
  return nb < nt ? nb : nt;
}

size_t conv3_wgrad_partial_floats(int cin, int cout, Grid3 g) {
  const int pairs = (cin < 16 ? 1 : cin / 16) * (cout / 16);
  return (size_t)pairs * wgrad_blocks(cin, cout, g) * 4 * 27 * 64 * 4;
}

int conv3_wgrad_partials(int cin, int cout, const uint16_t* x, const uint16_t* dy, const uint16_t* ymask,
                         float* partials, Grid3 g, hipStream_t s) {
  const int nb = wgrad_blocks(cin, cout, g);
  const int pairs = (cin < 16 ? 1 : cin / 16) * (cout / 16);
  f32x4* p = reinterpret_cast<f32x4*>(partials);
#define FE_CASE(a, b)                                                                                          \
  if (cin == a && cout == b) {                                                                                 \
    hipLaunchKernelGGL((k_wgrad<a, b>), dim3(nb, pairs), dim3(256), 0, s, x, dy, ymask, p, g);                \
    return nb * 4;                                                                                             \
  }
  FE_NN_CONV_SHAPES(FE_CASE)
#undef FE_CASE
  return 0;
}

void conv3_wgrad_reduce(int cin, int cout, const float* partials, int nsets, float* dw, hipStream_t s) {
  const f32x4* p = reinterpret_cast<const f32x4*>(partials);
#define FE_CASE(a, b)                                                                                 \
  if (cin == a && cout == b) {                                                                        \
    const int pairs = (a < 16 ? 1 : a / 16) * (b / 16);                                               \
    hipLaunchKernelGGL((k_wgrad_reduce<a, b>), dim3(pairs * 27), dim3(64 * kWgradSlices), 0, s, p, nsets, dw); \
    return;                                                                                           \
  }
  FE_NN_CONV_SHAPES(FE_CASE)
#undef FE_CASE
}

}  // namespace nn
}  // namespace fe
