// Internal interface of the U-Net prior kernels (unet.hip) for the C ABI layer.
// The 3x3x3 convolutions are the CNN kernels of cnn.h; these are the pieces
// the U-Net adds: 2x2x2 max pooling, the 2x2x2 stride-2 transposed
// convolution, and batch normalisation.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace clampk {

// Transposed convolution of a coarse tensor (nvol x nz x ny x nx, 32
// channels) to the fine grid (2 nz x 2 ny x 2 nx) plus bias and skip:
// out[2z+a][2y+b][2x+c][co] = bias[co] + skip[..][co] + sum_ci in[z][y][x][ci] W[4a+2b+c][ci][co].
struct UpArgs {
    int nvol, nz, ny, nx;    // coarse sizes
    const uint16_t* in;      // bf16 [voxel][32], coarse
    const uint16_t* wf;      // bf16 weight fragments [8][2][64][8] (unet_prep_up)
    const float* bias;       // fp32 [32]
    const uint16_t* skip;    // bf16 [voxel][32], fine
    uint16_t* out;           // bf16 [voxel][32], fine
};

// 2x2x2 max pooling of bf16 [voxel][32] (fine sizes, each even).
hipError_t unet_pool(const uint16_t* in, uint16_t* out, int nvol, int nz, int ny, int nx, hipStream_t st);
hipError_t unet_upconv(const UpArgs& a, hipStream_t st);
// MFMA weight fragments of a transposed convolution from fp32 W[8][32][32].
hipError_t unet_prep_up(const float* W, uint16_t* wf, hipStream_t st);
// Evaluation-mode batch normalisation folded into the bias-free convolution
// before it: wout = W s, bout = beta - mean s, s = gamma / sqrt(var + eps),
// per output channel (W: fp32 [27][cin][32]).
hipError_t unet_fold_bn(const float* W, const float* gamma, const float* beta, const float* mean, const float* var,
                        int cin, float* wout, float* bout, hipStream_t st);

constexpr float kBnEps = 1e-5f;

}  // namespace clampk
