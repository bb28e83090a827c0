// Internal interface of the CNN prior kernels (cnn.hip) for the C ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace clampk {

// Epilogues of the convolution: RELU stores ReLU(y + b); FINAL the one-channel
// output layer x + m (y + b) in fp32; DGRAD the backward-data product masked
// by the ReLU pattern of relu_src; RAW stores y unchanged (pre-activations
// before batch normalisation, or a backward-data product through a layer
// input that is no ReLU output).
enum ConvEpi { EPI_RELU = 0, EPI_FINAL = 1, EPI_DGRAD = 2, EPI_RAW = 3 };

struct ConvArgs {
    int nvol, nz, ny, nx;          // nx a multiple of 32
    int tiles_x, tiles_y;          // output tiles of 32 x-voxels and 16 rows (set by cnn_conv)
    int span;                      // output tile-slices per block (set by cnn_conv)
    const uint16_t* in;            // bf16 [voxel][CIN]
    const uint16_t* wq;            // bf16 weight fragments [9][kQ][2][32][8] (cnn_prep)
    const float* bias;             // fp32 [32] (EPI_RELU, EPI_FINAL)
    uint16_t* out;                 // bf16 [voxel][32] (EPI_RELU, EPI_DGRAD)
    float* out_f32;                // fp32 [voxel] (EPI_FINAL)
    const float* xin;              // fp32 [voxel] residual input (EPI_FINAL), the input (first layer)
    const float* scale;            // device scalar m of the output (EPI_FINAL), of the input (first layer); NULL = 1
    const uint16_t* relu_src;      // bf16 [voxel][32]: ReLU mask source (EPI_DGRAD)
};

struct WgradArgs {
    int nvol, nz, ny, nx;          // nx a multiple of 32
    int tiles_x, tiles_y;          // item tiles of 32 x-voxels and 8 rows (set by cnn_wgrad)
    int zc, zchunks, items;        // range slices per item, chunks per volume, items (set by cnn_wgrad)
    const uint16_t* act;           // bf16 [voxel][CA]: the layer input
    const uint16_t* g;             // bf16 [voxel][CG]: the gradient of the layer output
    float* part;                   // fp32 [2 * grid][28][32][32] partial sums (cnn_wgrad_part_bytes)
};

// cin = 1 with EPI_RELU: the first layer from the fp32 volume (xin, scale;
// weights from cnn_prep_first); cin = 8 or 32: bf16 inputs of that many
// channels.
hipError_t cnn_conv(int cin, int epi, ConvArgs a, hipStream_t st);
// First-layer weight fragments of k_conv_first (2048 bytes) from W [27][1][32].
hipError_t cnn_prep_first(const float* W, uint16_t* wq, hipStream_t st);
size_t cnn_wq_elems(int cinp);
hipError_t cnn_pack(const float* x, const float* scale, long nvox, uint16_t* x8, hipStream_t st);
int cnn_reduce_blocks(long nvox);
hipError_t cnn_mean(const float* x, long nvox, double* part, float* mean, hipStream_t st);
hipError_t cnn_loss(const float* out, const float* target, long nvox, uint16_t* g8, double* part, double* loss,
                    hipStream_t st);
int cnn_wgrad_grid();
size_t cnn_wgrad_part_bytes();
// Weight gradient gw[27][cin][cout] and bias gradient gb[cout] of one layer.
hipError_t cnn_wgrad(int ca, int cg, WgradArgs a, int cin, int cout, float* gw, float* gb, hipStream_t st);
// Adam step with gradient-norm clipping; clip: device float[kClipFloats],
// 8-byte aligned: the state clip[0..1] (zeroed with the parameters, see
// k_grad_clip), then kNormBlocks float64 partial sums of the squared norm.
constexpr int kNormBlocks = 64;
constexpr int kClipFloats = 2 + 2 * kNormBlocks;
hipError_t cnn_adam(float* p, float* m, float* v, const float* g, int n, float lr, int step, float* clip,
                    hipStream_t st);
// Weight fragments of a layer for the forward (wq, cinp input channels) and
// backward-data (wqd, coutp input channels; NULL to skip) convolutions and the
// padded bias.
hipError_t cnn_prep(const float* W, const float* b, int cin, int cout, int cinp, int coutp, uint16_t* wq,
                    uint16_t* wqd, float* bias32, hipStream_t st);

}  // namespace clampk
