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

// Backward passes of the transposed convolution (sizes of the coarse side).
struct UpBwdArgs {
    int nvol, nz, ny, nx;       // coarse sizes
    const uint16_t* g;          // bf16 [voxel][32], fine: gradient at the output
    const uint16_t* wt;         // transposed weight fragments (unet_prep_up, transposed = 1)
    const uint16_t* relu_src;   // bf16 coarse ReLU-mask source of the input gradient, or NULL
    const uint16_t* in;         // bf16 coarse input of the forward pass (weight gradient)
    uint16_t* out;              // bf16 coarse input gradient
};

// 2x2x2 max pooling of bf16 [voxel][32] (fine sizes, each even).
hipError_t unet_pool(const uint16_t* in, uint16_t* out, int nvol, int nz, int ny, int nx, hipStream_t st);
hipError_t unet_upconv(const UpArgs& a, hipStream_t st);
// MFMA weight fragments of a transposed convolution from fp32 W[8][32][32],
// for the forward product (transposed = 0) or the backward-data one (1).
hipError_t unet_prep_up(const float* W, int transposed, uint16_t* wf, hipStream_t st);
// Evaluation-mode batch normalisation folded into the bias-free convolution
// before it: wout = W s, bout = beta - mean s, s = gamma / sqrt(var + eps),
// per output channel (W: fp32 [27][cin][32]).
hipError_t unet_fold_bn(const float* W, const float* gamma, const float* beta, const float* mean, const float* var,
                        int cin, float* wout, float* bout, hipStream_t st);

constexpr float kBnEps = 1e-5f;
constexpr double kBnMomentum = 0.1;

// Training passes.
// Per-channel float64 sums of a bf16 [nvox][32] tensor into block partials
// (mode 0: x and x^2 of X; mode 1: dy and dy xhat with dy = X, xhat = (Y -
// mean) rstd); returns the number of partials through *blocks.
hipError_t unet_chan_sums(int mode, const uint16_t* X, const uint16_t* Y, const float* mean, const float* rstd,
                          long nvox, double* part, int* blocks, hipStream_t st);
size_t unet_chan_part_bytes();
// Reduction of the partials over m voxels (see k_chan_finalize): mode 0
// batch statistics (mean, rstd, A, B, running mean and variance), mode 1
// backward (dgamma -> out0, dbeta -> out1, coefficients A, B, C), mode 2 the
// plain sum -> out0.
hipError_t unet_chan_finalize(int mode, const double* part, int blocks, long m, const float* gamma, const float* beta,
                              float* mean, float* rstd, float* A, float* B, float* C, float* run_mean,
                              float* run_var, float* out0, float* out1, hipStream_t st);
// out = bf16([ReLU](A x + B y + C)) per channel (Y may be NULL: no B y term).
hipError_t unet_affine(const uint16_t* X, const uint16_t* Y, const float* A, const float* B, const float* C, int relu,
                       long nvox, uint16_t* out, hipStream_t st);
// de = [e > 0] (dp routed to each window's first maximum + dskip) (fine sizes).
hipError_t unet_pool_bwd(const uint16_t* e, const uint16_t* dp, const uint16_t* dskip, uint16_t* de, int nvol, int nz,
                         int ny, int nx, hipStream_t st);
hipError_t unet_upconv_dgrad(const UpBwdArgs& a, hipStream_t st);
// dW[8][32][32] into gw (fp32) through part (unet_upwgrad_part_bytes).
hipError_t unet_upconv_wgrad(const UpBwdArgs& a, float* part, float* gw, hipStream_t st);
size_t unet_upwgrad_part_bytes();

}  // namespace clampk
