// fsl_mlp.h -- sizes of the learned interface estimator and its launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fsl_kernels.h"

namespace fsl {

// FP32 parameter vector: W1[64][27], b1[64], W2[64][64], b2[64], W3[4][64], b3[4]
constexpr int MLP_OFF_W1 = 0;
constexpr int MLP_OFF_B1 = MLP_OFF_W1 + 64 * 27;
constexpr int MLP_OFF_W2 = MLP_OFF_B1 + 64;
constexpr int MLP_OFF_B2 = MLP_OFF_W2 + 64 * 64;
constexpr int MLP_OFF_W3 = MLP_OFF_B2 + 64;
constexpr int MLP_OFF_B3 = MLP_OFF_W3 + 4 * 64;
constexpr int MLP_NPARAM = MLP_OFF_B3 + 4;  // 6212

// packed BF16 operand copies: W1p[64][32], W2p[64][64], W3p[16][64], W2t[64][64], W3t[64][16]
constexpr int MLP_W2P = 64 * 32;
constexpr int MLP_W3P = MLP_W2P + 64 * 64;
constexpr int MLP_W2T = MLP_W3P + 16 * 64;
constexpr int MLP_W3T = MLP_W2T + 64 * 64;
constexpr int MLP_PACK_SIZE = MLP_W3T + 64 * 16;  // 12288

void mlp_pack(const float *P, uint16_t *pk, hipStream_t st);
void mlp_grad(const float *X, const float *T, const int32_t *idx, int nbatch, float inv_n, const float *P,
              const uint16_t *pk, int groups_per_wave, float *partial, float *partial_loss, int nwaves,
              float *grad, float *loss, hipStream_t st);
// one Adam step on a batch: gradient partials, then the fused update (sum,
// Adam, BF16 copies, batch loss)
void mlp_train_step(const float *X, const float *T, const int32_t *idx, int nbatch, float inv_n, float *P,
                    float *m, float *v, uint16_t *pk, int groups_per_wave, float *partial, float *partial_loss,
                    int nwaves, float lr, float b1, float b2, float eps, float c1, float c2, float *loss,
                    hipStream_t st);
void mlp_infer(const float *X, int n, const float *P, const uint16_t *pk, float *Y, hipStream_t st);
void fd_stencils(const float *X, int n, float *Y, hipStream_t st);
void stencil_fill(const double *P, int n, int ss, float *X, hipStream_t st);
template <class R>
void launch_geom_mlp(const Dev &d, int which, int blocks, const float *P, const uint16_t *pk, hipStream_t st);

}  // namespace fsl
