// Internal interface of the proposal network (kernels in k_cnn.hip).
//
// Network: 64 x 64 input; four 3 x 3 convolutions (zero padding, bias,
// ReLU) with 1 -> 32 -> 64 -> 128 -> 128 channels, each followed by a 2 x 2
// max pool; a fully connected layer from the 128 x 4 x 4 features to the L
// library orientations; softmax cross-entropy.  All arrays NCHW, FP32.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ebsd {
namespace cnn {

constexpr int kInSize = 64;
constexpr int kChannels[4] = {32, 64, 128, 128};
constexpr int kFeatures = 128 * 4 * 4;

// Offsets (in floats) of every tensor in the flat parameter vector:
// conv_i.w [co][ci][3][3], conv_i.b [co], fc.w [L][features], fc.b [L].
struct Layout {
  int64_t conv_w[4], conv_b[4], fc_w, fc_b, total;
  int classes;
};
Layout layout_of(int n_classes);

// The convolution weights in tap-major rows, wt_i[o][t ci + c] = w_i[o][c][t]
// (t = 3 dy + dx), layers one after another: offset of layer i and the total.
constexpr int64_t tap_weights_offset(int i) {
  int64_t off = 0;
  for (int l = 0, ci = 1; l < i; ci = kChannels[l], ++l) off += (int64_t)kChannels[l] * ci * 9;
  return off;
}
constexpr int64_t kTapWeights = tap_weights_offset(4);

// Activations of a batch: p[i] conv i output after ReLU and the pool,
// arg[i] the gradient positions of its pool, g[i] gradient at conv i's
// output (through ReLU), dp[i] gradient at p[i]; logits and their gradient
// dz; wt the tap-major copy of the convolution weights and the split
// halves of the weights for inference.
struct Acts {
  uint8_t* arg[4];  // per pooled output: the quad position its gradient goes to (4: none)
  float* p[4];
  float* g[4];  // gradient maps of layers 1..3 (g[0] is never formed)
  float* dp[4];
  float* logits;
  float* dz;
  float* wt;
  // split inference: BF16 halves of wt (layer i's rows at 2 x its offset) and
  // of the fc weights, rows interleaving groups of 8 hi and 8 lo halves
  unsigned short* wts;
  unsigned short* fcs;
};

hipError_t init_params(float* params, const Layout& lay, uint64_t seed, hipStream_t st);
// Weights in the forms the products read: the tap-major copy act.wt and,
// with split, the BF16 halves of it and of the fc weights.  Once per
// parameter version, before forward / backward.
hipError_t prepare(const float* params, const Layout& lay, const Acts& act, bool split, hipStream_t st);
// Each convolution writes its pooled map act.p; train: also the gradient
// positions act.arg that the backward pass needs.  split: the products take
// BF16 hi + lo halves of their FP32 operands, three products per tile (with
// train, the fc's only: the convolutions, whose outputs decide the ReLU and
// pool choices, stay FP32).
hipError_t forward(const float* params, const Layout& lay, const float* x, int64_t bsz, const Acts& act,
                   hipStream_t st, bool train = true, bool split = false);
// Gradient of the mean cross-entropy into grad (all of it overwritten), from
// act as the training forward pass on the same parameters left it;
// part: split-K scratch of part_floats floats; loss_row: [bsz] doubles.
// split: the products take BF16 split operands.
hipError_t backward(const float* params, const Layout& lay, const float* x, const int32_t* labels, int64_t bsz,
                    const Acts& act, float* grad, float* part, size_t part_floats, double* loss_row, float* loss,
                    hipStream_t st, bool split = false);
hipError_t adam(float* params, const float* grad, float* m, float* v, int64_t n, int64_t step, float lr,
                hipStream_t st);

// Training data: orientation and pattern centre of samples first .. first +
// bsz - 1, noise + binning of projected patterns, nearest-library labels.
hipError_t sample_setup(int64_t first, int64_t bsz, uint64_t seed, double pcx, double pcy, double pcz,
                        double max_off_frac, double* q, double* pc, hipStream_t st);
hipError_t noise_bin(const float* clean, int n, int64_t bsz, int64_t first, uint64_t seed, float counts, float snr,
                     int noisy, float* x, hipStream_t st);
hipError_t noise_bin(const __bf16* clean, int n, int64_t bsz, int64_t first, uint64_t seed, float counts,
                     float snr, int noisy, float* x, hipStream_t st);
hipError_t nearest_library(const double* q, int64_t bsz, const double* lib, int l, int32_t* label,
                           hipStream_t st);
hipError_t topk(const float* z, int64_t rows, int l, int k, int32_t* idx, hipStream_t st);

}  // namespace cnn
}  // namespace ebsd
