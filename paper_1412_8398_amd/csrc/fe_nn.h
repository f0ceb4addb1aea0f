// Warm-start U-Net: device helpers and launchers (bf16 storage, fp32 accumulation).
//
// Activations are channel-last, [sample][z][y][x][C] bf16, periodic in z, y, x.
// A 3^3 convolution is an implicit GEMM on the matrix cores: for an output
// voxel v and output channel o,
//   y[v, o] = b[o] + sum_{t < 27} sum_c x[v + off(t), c] w[t, c, o],
//   t = 9 (dz+1) + 3 (dy+1) + (dx+1),
// computed with v_mfma_f32_16x16x32_bf16: the A operand is 16 output channels
// x 32 reduction indices (weights, pre-packed per lane), the B operand is 32
// reduction indices x 16 voxels along x (input halo tile staged in LDS).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fe {
namespace nn {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;
typedef __attribute__((ext_vector_type(4))) uint32_t u32x4;

__host__ __device__ inline float bf2f(uint16_t h) {
  union {
    uint32_t u;
    float f;
  } c;
  c.u = (uint32_t)h << 16;
  return c.f;
}

// round to nearest even (finite inputs)
__host__ __device__ inline uint16_t f2bf(float f) {
  union {
    uint32_t u;
    float f;
  } c;
  c.f = f;
  const uint32_t u = c.u + 0x7fffu + ((c.u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

struct Grid3 {
  int nx, ny, nz, nb;  // grid and number of samples
  __host__ __device__ long long voxels() const { return (long long)nx * ny * nz * nb; }
};

// Output tile of the convolution kernels: 16 (x) x 4 (y) x 4 (z) voxels, one
// z slice per wavefront.
constexpr int TX = 16, TY = 4, TZ = 4;
constexpr int HX = TX + 2, HY = TY + 2, HZ = TZ + 2, HV = HX * HY * HZ;

__host__ __device__ constexpr int conv_cch(int cin) { return cin % 32 == 0 ? 32 : (cin % 16 == 0 ? 16 : 8); }
// Reduction steps of 32 per channel chunk.  The 9 (dz, dx) tap columns are
// dealt to the 32 / cch tap slots of a step in groups; each group takes 3
// steps, dy = -1, 0, +1, so a wavefront keeps a window of TY + 2 input rows
// in registers and reads each from LDS once per group (instead of once per
// output row and step).  Slots beyond the 9 columns carry zero weights.
__host__ __device__ constexpr int conv_groups(int cin) { return (9 + 32 / conv_cch(cin) - 1) / (32 / conv_cch(cin)); }
__host__ __device__ constexpr int conv_ksteps(int cin) { return 3 * conv_groups(cin); }
// packed weights: [chunk][kstep][out tile][lane] x 8 bf16 (16 bytes)
__host__ __device__ constexpr long long packed_elems(int cin, int cout) {
  return (long long)(cin / conv_cch(cin)) * conv_ksteps(cin) * (cout / 16) * 64 * 8;
}

__host__ __device__ inline int conv_tiles(const Grid3& g) {
  return ((g.nx + TX - 1) / TX) * ((g.ny + TY - 1) / TY) * ((g.nz + TZ - 1) / TZ) * g.nb;
}

// ---- launchers (fe_nn_conv.hip) ----
// y = act(conv3(x, w) + b); with mask non-null the input is x * (mask > 0)
// elementwise (mask has the input's shape): the masked gradient of a relu.
void conv3_forward(int cin, int cout, const uint16_t* x, const uint16_t* mask, const uint16_t* wpack,
                   const float* bias, int relu, uint16_t* y, Grid3 g, hipStream_t s);
// y = act(conv3([up2(coarse), skip], w) + b): the concatenation of the
// nearest upsampling of coarse (ca channels, grid g halved) and skip
// (cin - ca channels, grid g), read in place (the decoder layers)
bool conv_cat_supported(int cin, int cout, int ca);
void conv3_forward_cat(int cin, int cout, int ca, const uint16_t* coarse, const uint16_t* skip, const uint16_t* wpack,
                       const float* bias, int relu, uint16_t* y, Grid3 g, hipStream_t s);
// Per-block partial weight gradients for dw[t][c][o] = sum_v x[v + off(t), c] G[v, o],
// G = dy * (ymask > 0) (ymask nullable); returns the number of partial sets.
int conv3_wgrad_partials(int cin, int cout, const uint16_t* x, const uint16_t* dy, const uint16_t* ymask,
                         float* partials, Grid3 g, hipStream_t s);
size_t conv3_wgrad_partial_floats(int cin, int cout, Grid3 g);
void conv3_wgrad_reduce(int cin, int cout, const float* partials, int nsets, float* dw, hipStream_t s);
bool conv_supported(int cin, int cout);

// ---- elementwise / reduction launchers (fe_nn_ops.hip) ----
void pack_weights(const float* w, int cin, int cout, int flip, uint16_t* out, hipStream_t s);
struct FeatTab {  // per sample
  float logE[256];  // log10(E) / 3
  float nu[256];    // 10 (nu - 0.3)
  float macro[8];   // eps_bar (tensor Voigt order), 2 pad
};
void features(const uint8_t* phase, const FeatTab* tabs, uint16_t* x0, Grid3 g, hipStream_t s);
void pool2(const uint16_t* x, int c, uint16_t* y, Grid3 fine, hipStream_t s);
void up_concat(const uint16_t* coarse, int ca, const uint16_t* skip, int cb, uint16_t* out, Grid3 fine, hipStream_t s);
// g_coarse[v] = sum of g_cat[child, 0:ca] over the 8 children (gradient of up)
void up_backward(const uint16_t* gcat, int ca, int cb, uint16_t* gcoarse, Grid3 fine, hipStream_t s);
// g[v] = g_pool[parent(v)] / 8 + g_cat[v, ca:ca+c] (gradient of an encoder output)
void pool_backward_add(const uint16_t* gpool, const uint16_t* gcat, int ca, int c, uint16_t* g, Grid3 fine,
                       hipStream_t s);
// bias gradient partials: per block sums of dy * (ymask > 0)
int bias_grad(const uint16_t* dy, const uint16_t* ymask, int c, float* partials, float* db, Grid3 g, hipStream_t s);

// head: p = d1 hw + hb (16 -> 6); per-sample sums of p (and of the target)
// Blocks per sample of head_stats / head_backward (their partial sums).
int head_blocks(Grid3 g);
int head_stats(const uint16_t* d1, const float* hw, const float* hb, const void* target, int target_bf16,
               double* partials, double* sums, Grid3 g, hipStream_t s);
// prediction eps = p - mean(p) + eps_bar, written as float [sample][6][N]
void head_predict(const uint16_t* d1, const float* hw, const float* hb, const double* sums, const FeatTab* tabs,
                  float* out, Grid3 g, hipStream_t s);
// training: loss partials, gradient of d1 (bf16) and head gradient partials
int head_backward(const uint16_t* d1, const float* hw, const float* hb, const double* sums, const FeatTab* tabs,
                  const void* target, int target_bf16, uint16_t* gd1, double* partials, double* out_loss,
                  float* ghw, float* ghb, Grid3 g, hipStream_t s);
void adam(float* theta, const float* grad, float* m, float* v, long long n, float lr, float b1, float b2, float eps,
          int t, hipStream_t s);

}  // namespace nn
}  // namespace fe
