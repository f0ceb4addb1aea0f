/* Learned warm start for the Lippmann-Schwinger iteration: a 3D U-Net that
 * maps a microstructure and its applied strain to a starting strain field.
 *
 * The paper's schemes (eqs. (9) and (16)) accept any initial strain field;
 * the iteration from a predicted field still stops on the same equilibrium
 * criterion, eq. (43), so the network changes the starting point and never
 * the converged answer.  The network itself is not part of the paper.
 *
 * Network (channel-last bf16 activations, fp32 accumulation on the matrix
 * cores, fp32 master weights):
 *   input (8 channels): log10(E(x)) / 3, 10 (nu(x) - 0.3), eps_bar (6, tensor
 *     Voigt order 11, 22, 33, 23, 13, 12) broadcast over the grid;
 *   encoder: two periodic 3^3 convolutions + relu per level, widths 16, 32,
 *     64, 128, 2x2x2 average pooling between levels;
 *   decoder: nearest 2x upsampling, concatenation [upsampled, skip], two
 *     3^3 convolutions + relu per level (192->64->64, 96->32->32, 48->16->16);
 *   head: 1x1 linear 16 -> 6, then the mean over the cell is replaced by
 *     eps_bar (the average strain of every admissible field is eps_bar, eq. (6)).
 *   loss: mean over samples, voxels and the 6 components of the squared
 *     difference to a target strain field.
 * Grid lengths must be multiples of 8 (three poolings).
 *
 * Parameters, canonical order (float32): for each of the 14 convolutions
 * enc1a 8->16, enc1b 16->16, enc2a 16->32, enc2b 32->32, enc3a 32->64,
 * enc3b 64->64, bota 64->128, botb 128->128, dec3a 192->64, dec3b 64->64,
 * dec2a 96->32, dec2b 32->32, dec1a 48->16, dec1b 16->16: weights
 * [27][c_in][c_out] (tap t = 9 (dz+1) + 3 (dy+1) + (dx+1), y[v] gets
 * x[v + (dz, dy, dx)] w[t]) then bias [c_out]; then head weights [16][6] and
 * head bias [6].  1,462,694 values.
 *
 * Memory: all pointers marked "device" are caller-owned device memory; the
 * network object owns its parameters, optimizer state and a workspace sized
 * for the largest batch it has seen.  Calls on one network are not
 * thread-safe.  Errors: negative status, nothing written; fe_last_error()
 * holds the reason.
 */
#ifndef FE_NN_H
#define FE_NN_H

#include "fe.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fe_unet fe_unet;

typedef struct {
  uint32_t struct_size; /* sizeof(fe_unet_config) */
  uint64_t seed;        /* He-normal initial weights from SplitMix64 (Box-Muller), zero biases */
  float lr;             /* Adam step size (default 1e-3) */
  float beta1, beta2;   /* Adam moment decays (0.9, 0.999) */
  float adam_eps;       /* Adam denominator offset (1e-8) */
  void* hip_stream;     /* hipStream_t; NULL = default stream */
} fe_unet_config;

/* One batch of samples on a common grid.  phase: device uint8 [batch][nz][ny][nx];
 * materials: host array [batch] (n_phases <= 256, E > 0, -1 < nu < 0.5);
 * macro_strain: host float64 [batch][6]. */
typedef struct {
  fe_grid grid;
  int32_t batch;
  const uint8_t* phase;
  const fe_materials* materials;
  const double* macro_strain;
} fe_unet_batch;

void fe_unet_config_default(fe_unet_config* cfg);
fe_status fe_unet_create(const fe_unet_config* cfg, fe_unet** out);
void fe_unet_destroy(fe_unet* net);
int64_t fe_unet_param_count(void);

/* Adam step size for the following fe_unet_train_step calls (> 0, finite). */
fe_status fe_unet_set_learning_rate(fe_unet* net, float lr);

/* host float32 [fe_unet_param_count()] in canonical order; set also resets the
 * Adam moments and step counter */
fe_status fe_unet_get_params(fe_unet* net, float* host_params);
fe_status fe_unet_set_params(fe_unet* net, const float* host_params);
/* gradient left by the last fe_unet_loss_grad / fe_unet_train_step */
fe_status fe_unet_get_grads(fe_unet* net, float* host_grads);

/* Predicted strain, device float32 [batch][6][nz][ny][nx] (the layout of
 * fe_solve's strain_init).  seconds (nullable): device time of the call. */
fe_status fe_unet_predict(fe_unet* net, const fe_unet_batch* b, void* strain_out, double* seconds);

/* Loss and gradient against a target strain, device [batch][6][nz][ny][nx] of
 * float32 (target_bf16 = 0) or bfloat16 (1).  fe_unet_train_step also applies
 * one Adam step.  loss (nullable) receives the loss before the step. */
fe_status fe_unet_loss_grad(fe_unet* net, const fe_unet_batch* b, const void* target, int32_t target_bf16,
                            double* loss);
fe_status fe_unet_train_step(fe_unet* net, const fe_unet_batch* b, const void* target, int32_t target_bf16,
                             double* loss);

/* Single periodic 3^3 convolution layers on device bf16 channel-last
 * tensors [batch][nz][ny][nx][c] (building blocks of the network, exposed for
 * testing).  Weights w: device float32 [27][c_in][c_out], bias: device float32
 * [c_out] (nullable).  Supported (c_in, c_out): those of the network.
 * Each call allocates and frees its own packed-weight buffer. */
typedef struct {
  int32_t nx, ny, nz, batch, c_in, c_out;
} fe_nn_conv_shape;

/* y = (relu ? max(.,0) : id)(conv3(x, w) + b), y: [..][c_out] */
fe_status fe_nn_conv3_forward(const fe_nn_conv_shape* s, const uint16_t* x, const float* w, const float* b,
                              int32_t relu, uint16_t* y, void* hip_stream);
/* A decoder layer on its concatenated input read in place:
 * y = (relu ? max(.,0) : id)(conv3([up2(coarse), skip], w) + b), where up2 is
 * the nearest upsampling to s's grid (coarse: [..][nz/2][ny/2][nx/2][c_coarse],
 * even nx, ny, nz) and skip: [..][c_in - c_coarse].  Equal, bit for bit, to
 * fe_nn_conv3_forward on the materialised concatenation.  Supported
 * (c_in, c_out, c_coarse): (48, 16, 32), (96, 32, 64), (192, 64, 128). */
fe_status fe_nn_conv3_forward_cat(const fe_nn_conv_shape* s, int32_t c_coarse, const uint16_t* coarse,
                                  const uint16_t* skip, const float* w, const float* b, int32_t relu, uint16_t* y,
                                  void* hip_stream);
/* dx = gradient of sum(dy * y) with respect to x for y = conv3(x, w), where dy
 * is first multiplied by (y_mask > 0) when y_mask is not NULL (the relu of a
 * layer whose output is y_mask).  dy, y_mask: [..][c_out]; dx: [..][c_in];
 * c_in must be a multiple of 16. */
fe_status fe_nn_conv3_backward_data(const fe_nn_conv_shape* s, const uint16_t* dy, const uint16_t* y_mask,
                                    const float* w, uint16_t* dx, void* hip_stream);
/* dw[t][c][o] = sum_v x[v + off(t)][c] G[v][o], db[o] = sum_v G[v][o] with
 * G = dy * (y_mask > 0) (or dy); dw: device float32 [27][c_in][c_out], db
 * (nullable): device float32 [c_out]. */
fe_status fe_nn_conv3_backward_weight(const fe_nn_conv_shape* s, const uint16_t* x, const uint16_t* dy,
                                      const uint16_t* y_mask, float* dw, float* db, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* FE_NN_H */
